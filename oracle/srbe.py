"""SRBE estimators for a given sample of Fourier modes (oracle, FP64).

Test infrastructure only (see the package docstring).

Sec. 3 of the paper.  For a fixed sample {k_l}, l = 1..P (integer triples m_l,
duplicates counted with multiplicity) every SRBE quantity is a deterministic
function, written out here:

* the deterministic set I = {(0, 0, 2 pi m_z / Lz) : 1 <= |m_z| <= M}   (after Eq. (25));
* G = sum over L_k \\ I of exp(-k^2/(4 alpha^2))                        (Eq. (27)),
  evaluated as prod_d theta_d - 1 - 2 sum_{m=1..M} exp(-(2 pi m/Lz)^2/(4 alpha^2))
  with theta_d = sum_{m in Z} exp(-pi^2 m^2/(alpha^2 L_d^2)) (the Gaussian over
  the lattice factorises per axis);
* b*_F (Eq. (24)): exact over I plus (G/P) sum_l 4 pi/(V k_l^2) Re(exp(-i k_l.R_j) S1(k_l));
* F*_F (Eq. (25)): the same split with S1 + S2.

The rest of b and of the ion forces (real space, slab) is exact, as in
``oracle.ewald``.  The charges follow from Eqs. (9)-(10) with b* in place of b
(Algorithm 1, charge update).

Energy (a reading: the paper gives no SRBE energy estimator): with A exact,

    E* = 1/2 Q^T A Q - b*^T Q + c*,

where c* is c of Eq. (5) with its ion-ion Fourier term replaced by the same
estimator, 1/2 [sum_I w_k |S1|^2 + (G/P) sum_l 4 pi/(V k_l^2) |S1(k_l)|^2].
Then F* = -grad_r E* at fixed Q and b* = -dE*/dQ at Q = 0 for the fixed sample,
which the tests check by finite differences.
"""

import numpy as np

from . import ewald, cp


def deterministic_modes(M):
    """Integer triples of I: (0, 0, m) for m = -M..-1, 1..M (2M modes)."""
    mz = np.concatenate([np.arange(-M, 0), np.arange(1, M + 1)])
    return np.stack([np.zeros_like(mz), np.zeros_like(mz), mz], axis=1)


def theta(alpha, L, tol=1e-300):
    """theta(L) = sum_{m in Z} exp(-pi^2 m^2 / (alpha^2 L^2)), summed until terms drop below tol."""
    s = 1.0
    m = 1
    while True:
        t = np.exp(-(np.pi * m / (alpha * L)) ** 2)
        if t < tol:
            break
        s += 2.0 * t
        m += 1
    return s


def normaliser_G(p):
    """Eq. (27): G = sum_{k in L_k \\ I} exp(-k^2/(4 alpha^2))."""
    prod = theta(p.alpha, p.Lx) * theta(p.alpha, p.Ly) * theta(p.alpha, p.Lz)
    mI = np.arange(1, p.M + 1)
    det = 2.0 * np.sum(np.exp(-((2.0 * np.pi * mI / p.Lz) ** 2) / (4.0 * p.alpha ** 2)))
    return prod - 1.0 - det


def mode_weights(p, kset):
    """Weights of the deterministic modes and of the sampled modes.

    Returns (mI, wI, mS, wS): on I, w = 4 pi exp(-k^2/(4 alpha^2))/(V k^2) (Eq. (24) first
    sum); for each sampled occurrence, w = (G/P) 4 pi/(V k^2) (second sum).
    """
    mI = deterministic_modes(p.M)
    kI = ewald.kvectors(p, mI)
    wI = ewald.ewald_weight(p, np.sum(kI ** 2, axis=1))
    mS = np.asarray(kset, dtype=np.int64).reshape(-1, 3)
    kS = ewald.kvectors(p, mS)
    Pn = len(mS)
    G = normaliser_G(p)
    wS = (G / Pn) * 4.0 * np.pi / (p.V * np.sum(kS ** 2, axis=1)) if Pn else np.zeros(0)
    return mI, wI, mS, wS


def _combined(p, kset):
    mI, wI, mS, wS = mode_weights(p, kset)
    return np.concatenate([mI, mS]), np.concatenate([wI, wS])


def srbe_b_fourier(p, kset, ion_pos, ion_q, ele_pos):
    """Eq. (24): b*_F,j = -sum_I w_k Re(e^{-ik.R_j} S1(k)) - (G/P) sum_l 4 pi/(V k_l^2) Re(e^{-ik_l.R_j} S1(k_l))."""
    ion_pos = np.asarray(ion_pos, dtype=np.float64).reshape(-1, 3)
    ele_pos = np.asarray(ele_pos, dtype=np.float64).reshape(-1, 3)
    m, w = _combined(p, kset)
    S1 = ewald.structure_factor(p, m, ion_pos, np.asarray(ion_q, dtype=np.float64))
    return -p.coulomb_k * ewald.fourier_potential(p, m, w * S1, ele_pos)


def srbe_force_fourier(p, kset, ion_pos, ion_q, ele_pos, Q):
    """Eq. (25): Fourier force on every ion with S = S1 + S2 (times coulomb_k)."""
    ion_pos = np.asarray(ion_pos, dtype=np.float64).reshape(-1, 3)
    ele_pos = np.asarray(ele_pos, dtype=np.float64).reshape(-1, 3)
    ion_q = np.asarray(ion_q, dtype=np.float64)
    m, w = _combined(p, kset)
    S = ewald.structure_factor(p, m, ion_pos, ion_q) + ewald.structure_factor(p, m, ele_pos, Q)
    return -p.coulomb_k * ion_q[:, None] * ewald.fourier_gradient_term(p, m, w * S, ion_pos)


def srbe_b(p, kset, ion_pos, ion_q, ele_pos):
    """b* for one sample: Eq. (24) Fourier part + exact slab and real-space parts (times coulomb_k)."""
    ion_pos = np.asarray(ion_pos, dtype=np.float64).reshape(-1, 3)
    ele_pos = np.asarray(ele_pos, dtype=np.float64).reshape(-1, 3)
    ion_q = np.asarray(ion_q, dtype=np.float64)
    bF = srbe_b_fourier(p, kset, ion_pos, ion_q, ele_pos) / p.coulomb_k
    bS = -(4.0 * np.pi / p.V) * ele_pos[:, 2] * (ion_q @ ion_pos[:, 2]) if p.slab else 0.0
    phi, _ = ewald.real_space(p, "ig", ele_pos, ion_pos, ion_q)
    return p.coulomb_k * (bF + bS - phi)


def srbe_ion_forces(p, kset, ion_pos, ion_q, ele_pos, Q):
    """F* on every ion: Eq. (25) + slab force (reading) + exact real space (times coulomb_k)."""
    ion_pos = np.asarray(ion_pos, dtype=np.float64).reshape(-1, 3)
    ele_pos = np.asarray(ele_pos, dtype=np.float64).reshape(-1, 3)
    ion_q = np.asarray(ion_q, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    F = srbe_force_fourier(p, kset, ion_pos, ion_q, ele_pos, Q) / p.coulomb_k
    if p.slab:
        Mz = ion_q @ ion_pos[:, 2] + Q @ ele_pos[:, 2]
        F[:, 2] -= (4.0 * np.pi / p.V) * ion_q * Mz
    _, gii = ewald.real_space(p, "ii", ion_pos, ion_pos, ion_q, same=True)
    _, gig = ewald.real_space(p, "ig", ion_pos, ele_pos, Q)
    F -= ion_q[:, None] * (gii + gig)
    return p.coulomb_k * F


def _real_chunk(n_src):
    """Targets per real-space chunk so that a chunk's pair arrays stay near 2^22 entries."""
    return max(1, (1 << 22) // max(n_src, 1))


def srbe_b_at(p, kset, ion_pos, ion_q, ele_pos, idx):
    """srbe_b at the electrodes ``idx`` only (same terms; for systems too large to do all)."""
    ion_pos = np.asarray(ion_pos, dtype=np.float64).reshape(-1, 3)
    ele_pos = np.asarray(ele_pos, dtype=np.float64).reshape(-1, 3)
    ion_q = np.asarray(ion_q, dtype=np.float64)
    tgt = ele_pos[np.asarray(idx)]
    m, w = _combined(p, kset)
    S1 = ewald.structure_factor(p, m, ion_pos, ion_q)
    bF = -ewald.fourier_potential(p, m, w * S1, tgt)
    bS = -(4.0 * np.pi / p.V) * tgt[:, 2] * (ion_q @ ion_pos[:, 2]) if p.slab else 0.0
    phi, _ = ewald.real_space(p, "ig", tgt, ion_pos, ion_q, chunk=_real_chunk(len(ion_pos)))
    return p.coulomb_k * (bF + bS - phi)


def srbe_ion_forces_at(p, kset, ion_pos, ion_q, ele_pos, Q, idx):
    """srbe_ion_forces on the ions ``idx`` only (same terms; for systems too large to do all)."""
    ion_pos = np.asarray(ion_pos, dtype=np.float64).reshape(-1, 3)
    ele_pos = np.asarray(ele_pos, dtype=np.float64).reshape(-1, 3)
    ion_q = np.asarray(ion_q, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    idx = np.asarray(idx)
    tgt, qt = ion_pos[idx], ion_q[idx]
    m, w = _combined(p, kset)
    S = ewald.structure_factor(p, m, ion_pos, ion_q) + ewald.structure_factor(p, m, ele_pos, Q)
    F = -qt[:, None] * ewald.fourier_gradient_term(p, m, w * S, tgt)
    if p.slab:
        Mz = ion_q @ ion_pos[:, 2] + Q @ ele_pos[:, 2]
        F[:, 2] -= (4.0 * np.pi / p.V) * qt * Mz
    _, gii = ewald.real_space(p, "ii", tgt, ion_pos, ion_q, exclude=idx, chunk=_real_chunk(len(ion_pos)))
    _, gig = ewald.real_space(p, "ig", tgt, ele_pos, Q, chunk=_real_chunk(len(ele_pos)))
    F -= qt[:, None] * (gii + gig)
    return p.coulomb_k * F


def srbe_ele_forces(p, kset, ion_pos, ion_q, ele_pos, Q):
    """Forces on the electrode atoms from the same estimator (used for the momentum check)."""
    ion_pos = np.asarray(ion_pos, dtype=np.float64).reshape(-1, 3)
    ele_pos = np.asarray(ele_pos, dtype=np.float64).reshape(-1, 3)
    ion_q = np.asarray(ion_q, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    m, w = _combined(p, kset)
    S = ewald.structure_factor(p, m, ion_pos, ion_q) + ewald.structure_factor(p, m, ele_pos, Q)
    F = -Q[:, None] * ewald.fourier_gradient_term(p, m, w * S, ele_pos)
    if p.slab:
        Mz = ion_q @ ion_pos[:, 2] + Q @ ele_pos[:, 2]
        F[:, 2] -= (4.0 * np.pi / p.V) * Q * Mz
    _, gig = ewald.real_space(p, "ig", ele_pos, ion_pos, ion_q)
    _, ggg = ewald.real_space(p, "gg", ele_pos, ele_pos, Q, same=True)
    F -= Q[:, None] * (gig + ggg)
    return p.coulomb_k * F


def srbe_constant(p, kset, ion_pos, ion_q):
    """c*: ion-ion real space + estimated ion-ion Fourier + ion self + ion slab (times coulomb_k)."""
    ion_pos = np.asarray(ion_pos, dtype=np.float64).reshape(-1, 3)
    ion_q = np.asarray(ion_q, dtype=np.float64)
    m, w = _combined(p, kset)
    S1 = ewald.structure_factor(p, m, ion_pos, ion_q)
    u_four = 0.5 * np.sum(w * np.abs(S1) ** 2)
    phi, _ = ewald.real_space(p, "ii", ion_pos, ion_pos, ion_q, same=True)
    u_real = 0.5 * ion_q @ phi
    _, ci = ewald.self_constants(p)
    u_self = -ci * np.sum(ion_q ** 2)
    u_slab = (2.0 * np.pi / p.V) * (ion_q @ ion_pos[:, 2]) ** 2 if p.slab else 0.0
    return p.coulomb_k * (u_real + u_four + u_self + u_slab)


def srbe_energy(p, A, kset, ion_pos, ion_q, ele_pos, Q, b=None):
    """E* = 1/2 Q^T A Q - b*^T Q + c* (reading described in the module docstring)."""
    b = srbe_b(p, kset, ion_pos, ion_q, ele_pos) if b is None else b
    Q = np.asarray(Q, dtype=np.float64)
    return 0.5 * Q @ (A @ Q) - b @ Q + srbe_constant(p, kset, ion_pos, ion_q)


def srbe_energy_parts(p, kset, ion_pos, ion_q, ele_pos, Q, modes=None):
    """E* split as U_c is in Eqs. (13), (16), (17): real, fourier, self, slab, total (times coulomb_k).

    The SRBE changes only the Fourier part, so each other part is the complete one:
      real    = 1/2 q.phi_ii + Q.phi_ig + 1/2 Q.phi_gg      (erfc kernels, r < rc, Eq. (13))
      self    = c_g sum Q^2 - c_i sum q^2                    (Eq. (17))
      slab    = (2 pi / V) (sum q z + sum Q Z)^2             (Eq. (17))
      fourier = 1/2 sum_all w |S2|^2 + sum_est w Re(S1 conj S2) + 1/2 sum_est w |S1|^2,
    the electrode-electrode Fourier term exact (A is), the ion-electrode and ion-ion ones
    over the deterministic modes and the sample (Eq. (24) and c*).  `modes` is the
    complete mode set of A (default: ewald.enumerate_modes).
    """
    ion_pos = np.asarray(ion_pos, dtype=np.float64).reshape(-1, 3)
    ele_pos = np.asarray(ele_pos, dtype=np.float64).reshape(-1, 3)
    ion_q = np.asarray(ion_q, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    modes = ewald.enumerate_modes(p) if modes is None else modes
    phi_ii, _ = ewald.real_space(p, "ii", ion_pos, ion_pos, ion_q, same=True)
    phi_ig, _ = ewald.real_space(p, "ig", ele_pos, ion_pos, ion_q)
    phi_gg, _ = ewald.real_space(p, "gg", ele_pos, ele_pos, Q, same=True)
    u_real = 0.5 * ion_q @ phi_ii + Q @ phi_ig + 0.5 * Q @ phi_gg
    k2 = np.sum(ewald.kvectors(p, modes) ** 2, axis=1)
    S2_all = ewald.structure_factor(p, modes, ele_pos, Q)
    u_gg = 0.5 * np.sum(ewald.ewald_weight(p, k2) * np.abs(S2_all) ** 2)
    m, w = _combined(p, kset)
    S1 = ewald.structure_factor(p, m, ion_pos, ion_q)
    S2 = ewald.structure_factor(p, m, ele_pos, Q)
    u_four = u_gg + np.sum(w * np.real(S1 * np.conj(S2))) + 0.5 * np.sum(w * np.abs(S1) ** 2)
    cg, ci = ewald.self_constants(p)
    u_self = cg * np.sum(Q ** 2) - ci * np.sum(ion_q ** 2)
    Mz = ion_q @ ion_pos[:, 2] + Q @ ele_pos[:, 2]
    u_slab = (2.0 * np.pi / p.V) * Mz ** 2 if p.slab else 0.0
    ke = p.coulomb_k
    out = dict(real=ke * u_real, fourier=ke * u_four, self=ke * u_self, slab=ke * u_slab)
    out["total"] = out["real"] + out["fourier"] + out["self"] + out["slab"]
    return out


def srbe_step(p, solver, kset, ion_pos, ion_q, ele_pos, ele_side, dpsi, Q_fixed=None):
    """One SRBE step without integration (Algorithm 1, steps 'compute b, update Q, compute forces').

    If Q_fixed is given the charges are not solved (fixed-charge mode).
    Returns a dict with b, Q, psibar, F (ions), E.
    """
    b = srbe_b(p, kset, ion_pos, ion_q, ele_pos)
    if Q_fixed is None:
        Q, psibar = solver.solve(ele_side, dpsi, b)
    else:
        Q = np.asarray(Q_fixed, dtype=np.float64)
        psibar = np.nan
    F = srbe_ion_forces(p, kset, ion_pos, ion_q, ele_pos, Q)
    E = srbe_energy(p, solver.A, kset, ion_pos, ion_q, ele_pos, Q, b=b)
    return dict(b=b, Q=Q, psibar=psibar, F=F, E=E)


def full_step(p, solver, ion_pos, ion_q, ele_pos, ele_side, dpsi, modes=None, Q_fixed=None):
    """The same outputs computed with the complete reciprocal sums (what SRBE estimates)."""
    modes = ewald.enumerate_modes(p) if modes is None else modes
    b = ewald.electrode_vector(p, ion_pos, ion_q, ele_pos, modes=modes)
    if Q_fixed is None:
        Q, psibar = solver.solve(ele_side, dpsi, b)
    else:
        Q = np.asarray(Q_fixed, dtype=np.float64)
        psibar = np.nan
    F, _ = ewald.forces(p, ion_pos, ion_q, ele_pos, Q, modes=modes)
    E = ewald.energy(p, ion_pos, ion_q, ele_pos, Q, modes=modes)["total"]
    return dict(b=b, Q=Q, psibar=psibar, F=F, E=E)
