"""Ewald decomposition with zero-padded slab correction (oracle, FP64).

Test infrastructure only (see the package docstring).

The system (Sec. 2): ions (point charges q_i at r_i) and fixed electrode atoms
carrying Gaussian charges Q_j of width eta (a length, Eq. (1)) at R_j, in the box
[0,Lx] x [0,Ly] x [0,H], periodic in x and y.  The z direction is padded to
Lz = lambda * H and treated as periodic with the Yeh-Berkowitz correction
(Eqs. (16)-(17)); V = Lx Ly Lz.

Every function here is a direct transcription of a definition in Sec. 2 with no
blocking or reordering beyond chunking a sum to bound memory:

* Eq. (12): 1/r = erf(alpha r)/r + erfc(alpha r)/r;
* Eq. (13): the real-space part U_N (ion-ion, ion-Gaussian, Gaussian-Gaussian
  kernels), images n in Z^2 x {0} (Z^3 in the fully periodic mode);
* Eq. (15): structure factors S(k) = sum_j q_j exp(i k.r_j);
* Eq. (16): U_F = 1/(2V) sum_{k in L_k} 4 pi/k^2 |S1+S2|^2 exp(-k^2/(4 alpha^2)),
  L_k = 2 pi Z^3 o L^-1 \\ {0};
* Eq. (17): U_corr (self terms and the k=0 slab term);  U_c = U_N + U_F - U_corr;
* Eq. (18): the electrode matrix A, Eq. (19): the vector b, so that
  U_c(Q) = 1/2 Q^T A Q - b^T Q + c (Eq. (5));
* Eq. (21): the Fourier force on the ions.

Readings (places where the printed formulas disagree with Eq. (17)):

* A's slab entry is printed (2 pi/V) Z_i Z_j in Eq. (18), but the Hessian of the
  slab term (2 pi/V)(sum q z + sum Q Z)^2 of Eq. (17) in Q is (4 pi/V) Z_i Z_j.
  We use 4 pi/V, the value that makes Eq. (5) hold.  Pinned by a finite-difference
  Hessian of ``energy``.
* b's slab entry is printed +(4 pi Z_j/V) sum q_i z_i in Eq. (19); b = -dU/dQ at
  Q = 0 gives -(4 pi Z_j/V) sum q_i z_i.  We use the minus sign.  Pinned by a
  finite-difference gradient of ``energy``.
* Eq. (19) adds +Delta psi to b; it is already carried by the Delta psi d term of
  Eq. (10) and is dropped here (any constant added to b leaves Q unchanged, which
  a test checks).
* Eqs. (21) and (25) omit the force of the slab (k = 0) term of Eq. (17); we
  include -(4 pi/V) q_i M_z e_z with M_z = sum q z + sum Q Z, the gradient of
  that term.

All Coulomb terms carry the factor ``coulomb_k`` (1 in the paper's units).
"""

from dataclasses import dataclass, replace

import numpy as np
from scipy.special import erfc

SQRT_PI = np.sqrt(np.pi)


@dataclass(frozen=True)
class Params:
    """Geometry and Ewald parameters.

    Lx, Ly, H: box; lam: zero-padding ratio (Lz = lam * H); alpha: splitting
    parameter; eta: Gaussian width (a length, Eq. (1)); rc: real-space cutoff;
    coulomb_k: Coulomb constant; M: number of deterministic k_z modes; P: batch
    size; kspace_tol: the full reciprocal sums keep every k with
    exp(-k^2/(4 alpha^2)) >= kspace_tol; slab: apply the Eq. (17) k=0 term (False
    means tin-foil 3-D periodic Ewald); periodic_z: real-space images also in z
    (fully periodic mode, used only by pins).
    """

    Lx: float
    Ly: float
    H: float
    lam: float = 3.0
    alpha: float = 3.0
    eta: float = 0.05
    rc: float = 1.2
    coulomb_k: float = 1.0
    M: int = 0
    P: int = 0
    kspace_tol: float = 1e-16
    slab: bool = True
    periodic_z: bool = False

    @property
    def Lz(self):
        return self.lam * self.H

    @property
    def L(self):
        return np.array([self.Lx, self.Ly, self.Lz])

    @property
    def V(self):
        return self.Lx * self.Ly * self.Lz

    def with_(self, **kw):
        return replace(self, **kw)


# ---------------------------------------------------------------- reciprocal space


def kvectors(p, m):
    """k = 2 pi m o L^-1 for integer triples m (shape (K, 3))."""
    return 2.0 * np.pi * np.asarray(m, dtype=np.float64) / p.L


def ewald_weight(p, k2):
    """4 pi exp(-k^2/(4 alpha^2)) / (V k^2): the weight of mode k in Eqs. (16), (18), (19)."""
    return 4.0 * np.pi * np.exp(-k2 / (4.0 * p.alpha ** 2)) / (p.V * k2)


def enumerate_modes(p, tol=None):
    """All m in Z^3 \\ {0} with exp(-|k|^2/(4 alpha^2)) >= tol (both signs of every mode)."""
    tol = p.kspace_tol if tol is None else tol
    k2max = 4.0 * p.alpha ** 2 * np.log(1.0 / tol)
    mmax = np.floor(np.sqrt(k2max) * p.L / (2.0 * np.pi)).astype(int)
    axes = [np.arange(-n, n + 1) for n in mmax]
    mx, my, mz = np.meshgrid(*axes, indexing="ij")
    m = np.stack([mx.ravel(), my.ravel(), mz.ravel()], axis=1)
    k2 = np.sum(kvectors(p, m) ** 2, axis=1)
    keep = (k2 > 0) & (k2 <= k2max)
    return m[keep]


def structure_factor(p, m, pos, q, chunk=4096, pchunk=65536):
    """Eq. (15): S(k) = sum_j q_j exp(i k.r_j) for every mode m (returns complex (K,)).

    Particles are taken pchunk at a time (their partial sums added in order), so the
    phase matrix stays small for large systems.
    """
    kv = kvectors(p, m)
    pos = np.asarray(pos)
    q = np.asarray(q)
    out = np.zeros(len(kv), dtype=np.complex128)
    for s in range(0, len(kv), chunk):
        for j in range(0, len(pos), pchunk):
            ph = pos[j:j + pchunk] @ kv[s:s + chunk].T
            out[s:s + chunk] += q[j:j + pchunk] @ np.exp(1j * ph)
    return out


def fourier_potential(p, m, coef, pos, chunk=2048):
    """sum_k Re(coef_k exp(-i k.r)) at each position (returns (N,))."""
    kv = kvectors(p, m)
    out = np.zeros(len(pos))
    for s in range(0, len(kv), chunk):
        e = np.exp(-1j * (np.asarray(pos) @ kv[s:s + chunk].T))
        out += np.real(e @ coef[s:s + chunk])
    return out


def fourier_gradient_term(p, m, coef, pos, chunk=2048):
    """sum_k k Im(coef_k exp(-i k.r)) at each position (returns (N, 3))."""
    kv = kvectors(p, m)
    out = np.zeros((len(pos), 3))
    for s in range(0, len(kv), chunk):
        e = np.exp(-1j * (np.asarray(pos) @ kv[s:s + chunk].T))
        out += np.imag(e * coef[s:s + chunk][None, :]) @ kv[s:s + chunk]
    return out


# ---------------------------------------------------------------- real space (Eq. (13))


def kernel_ion_ion(p, r):
    return erfc(p.alpha * r) / r


def kernel_ion_gauss(p, r):
    return (erfc(p.alpha * r) - erfc(r / p.eta)) / r


def kernel_gauss_gauss(p, r):
    return (erfc(p.alpha * r) - erfc(r / (np.sqrt(2.0) * p.eta))) / r


def _derf_c(a, r):
    """d/dr [erfc(a r)/r]."""
    return -erfc(a * r) / r ** 2 - 2.0 * a / SQRT_PI * np.exp(-(a * r) ** 2) / r


def dkernel_ion_ion(p, r):
    return _derf_c(p.alpha, r)


def dkernel_ion_gauss(p, r):
    return _derf_c(p.alpha, r) - _derf_c(1.0 / p.eta, r)


def dkernel_gauss_gauss(p, r):
    return _derf_c(p.alpha, r) - _derf_c(1.0 / (np.sqrt(2.0) * p.eta), r)


KERNELS = {
    "ii": (kernel_ion_ion, dkernel_ion_ion),
    "ig": (kernel_ion_gauss, dkernel_ion_gauss),
    "gg": (kernel_gauss_gauss, dkernel_gauss_gauss),
}


def image_shifts(p):
    """Shifts n o l covering every image closer than rc, for positions inside the box."""
    ns = []
    lengths = [p.Lx, p.Ly] + ([p.Lz] if p.periodic_z else [])
    for Ld in lengths:
        nmax = 1 + int(np.floor(p.rc / Ld))
        ns.append(np.arange(-nmax, nmax + 1))
    if not p.periodic_z:
        ns.append(np.array([0]))
    g = np.meshgrid(*ns, indexing="ij")
    n = np.stack([a.ravel() for a in g], axis=1)
    return n * p.L


def wrap_xy(p, pos):
    """Map x, y into [0, L) (z is left alone unless the mode is fully periodic)."""
    pos = np.array(pos, dtype=np.float64, copy=True)
    pos[:, 0] = np.mod(pos[:, 0], p.Lx)
    pos[:, 1] = np.mod(pos[:, 1], p.Ly)
    if p.periodic_z:
        pos[:, 2] = np.mod(pos[:, 2], p.Lz)
    return pos


def real_space(p, kind, tgt, src, src_q, same=False, chunk=512, exclude=None):
    """Real-space potential and field of Eq. (13) kernels.

    phi_t = sum_s sum_n q_s K(|r_t - r_s - n o l|) over |.| < rc, excluding the
    s = t, n = 0 term when ``same`` (the sources are the targets), or the
    s = exclude[t], n = 0 term when ``exclude`` (one source index per target) is
    given.  grad_t = d phi_t / d r_t.
    Returns (phi (T,), grad (T, 3)).
    """
    if same:
        exclude = np.arange(len(tgt))
    K, dK = KERNELS[kind]
    tgt = wrap_xy(p, tgt)
    src = wrap_xy(p, src)
    src_q = np.asarray(src_q, dtype=np.float64)
    phi = np.zeros(len(tgt))
    grad = np.zeros((len(tgt), 3))
    if not p.periodic_z and p.rc <= 0.5 * min(p.Lx, p.Ly):
        # minimum image: with rc <= L/2 only the nearest periodic copy can lie within rc
        for t0 in range(0, len(tgt), chunk):
            tb = tgt[t0:t0 + chunk]
            d = tb[:, None, :] - src[None, :, :]
            d[..., 0] -= p.Lx * np.round(d[..., 0] / p.Lx)
            d[..., 1] -= p.Ly * np.round(d[..., 1] / p.Ly)
            r = np.sqrt(np.sum(d * d, axis=2))
            mask = r < p.rc
            if exclude is not None:
                mask[np.arange(len(tb)), exclude[t0:t0 + len(tb)]] = False
            rr = np.where(mask, r, 1.0)
            kv = np.where(mask, K(p, rr), 0.0)
            dk = np.where(mask, dK(p, rr), 0.0)
            phi[t0:t0 + chunk] += kv @ src_q
            grad[t0:t0 + chunk] += np.einsum("ts,tsd->td", dk * src_q[None, :] / rr, d)
        return phi, grad
    shifts = image_shifts(p)
    for t0 in range(0, len(tgt), chunk):
        tb = tgt[t0:t0 + chunk]
        for sh in shifts:
            d = tb[:, None, :] - src[None, :, :] - sh[None, None, :]
            r = np.sqrt(np.sum(d * d, axis=2))
            mask = r < p.rc
            if exclude is not None and not np.any(sh):
                mask[np.arange(len(tb)), exclude[t0:t0 + len(tb)]] = False
            rr = np.where(mask, r, 1.0)
            kv = np.where(mask, K(p, rr), 0.0)
            dk = np.where(mask, dK(p, rr), 0.0)
            phi[t0:t0 + chunk] += kv @ src_q
            grad[t0:t0 + chunk] += np.einsum("ts,tsd->td", dk * src_q[None, :] / rr, d)
    return phi, grad


# ---------------------------------------------------------------- energy (Eqs. (13)-(17))


def self_constants(p):
    """(1/(sqrt(2 pi) eta) - alpha/sqrt(pi), alpha/sqrt(pi)) of Eq. (17)."""
    return 1.0 / (np.sqrt(2.0 * np.pi) * p.eta) - p.alpha / SQRT_PI, p.alpha / SQRT_PI


def energy(p, ion_pos, ion_q, ele_pos, Q, modes=None):
    """U_c = U_N + U_F - U_corr (Eqs. (13), (16), (17)), computed from its definition.

    Returns a dict of components (all scaled by coulomb_k): real, fourier, self, slab, total.
    """
    ion_pos = np.asarray(ion_pos, dtype=np.float64).reshape(-1, 3)
    ele_pos = np.asarray(ele_pos, dtype=np.float64).reshape(-1, 3)
    ion_q = np.asarray(ion_q, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    modes = enumerate_modes(p) if modes is None else modes
    # U_N
    u_real = 0.0
    if len(ion_pos):
        phi_ii, _ = real_space(p, "ii", ion_pos, ion_pos, ion_q, same=True)
        u_real += 0.5 * ion_q @ phi_ii
    if len(ion_pos) and len(ele_pos):
        phi_ig, _ = real_space(p, "ig", ele_pos, ion_pos, ion_q)
        u_real += Q @ phi_ig
    if len(ele_pos):
        phi_gg, _ = real_space(p, "gg", ele_pos, ele_pos, Q, same=True)
        u_real += 0.5 * Q @ phi_gg
    # U_F
    pos = np.concatenate([ion_pos, ele_pos])
    qq = np.concatenate([ion_q, Q])
    S = structure_factor(p, modes, pos, qq)
    k2 = np.sum(kvectors(p, modes) ** 2, axis=1)
    u_four = 0.5 * np.sum(ewald_weight(p, k2) * np.abs(S) ** 2)
    # -U_corr
    cg, ci = self_constants(p)
    u_self = cg * np.sum(Q ** 2) - ci * np.sum(ion_q ** 2)
    Mz = ion_q @ ion_pos[:, 2] + Q @ ele_pos[:, 2]
    u_slab = (2.0 * np.pi / p.V) * Mz ** 2 if p.slab else 0.0
    ke = p.coulomb_k
    out = dict(real=ke * u_real, fourier=ke * u_four, self=ke * u_self, slab=ke * u_slab)
    out["total"] = sum(out.values())
    return out


def forces(p, ion_pos, ion_q, ele_pos, Q, modes=None):
    """-grad U_c with respect to every particle (Eq. (21) plus real-space and slab terms).

    Returns (F_ion (N_ion, 3), F_ele (N_ele, 3)).
    """
    ion_pos = np.asarray(ion_pos, dtype=np.float64).reshape(-1, 3)
    ele_pos = np.asarray(ele_pos, dtype=np.float64).reshape(-1, 3)
    ion_q = np.asarray(ion_q, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    modes = enumerate_modes(p) if modes is None else modes
    pos = np.concatenate([ion_pos, ele_pos])
    qq = np.concatenate([ion_q, Q])
    S = structure_factor(p, modes, pos, qq)
    k2 = np.sum(kvectors(p, modes) ** 2, axis=1)
    coef = ewald_weight(p, k2) * S
    # Fourier (Eq. (21), applied to every particle)
    g = fourier_gradient_term(p, modes, coef, pos)
    F = -qq[:, None] * g
    # slab term of Eq. (17)
    if p.slab:
        Mz = qq @ pos[:, 2]
        F[:, 2] -= (4.0 * np.pi / p.V) * qq * Mz
    # real space
    ni = len(ion_pos)
    if ni:
        _, gii = real_space(p, "ii", ion_pos, ion_pos, ion_q, same=True)
        F[:ni] -= ion_q[:, None] * gii
        if len(ele_pos):
            _, gig = real_space(p, "ig", ion_pos, ele_pos, Q)
            F[:ni] -= ion_q[:, None] * gig
            _, ggi = real_space(p, "ig", ele_pos, ion_pos, ion_q)
            F[ni:] -= Q[:, None] * ggi
    if len(ele_pos):
        _, ggg = real_space(p, "gg", ele_pos, ele_pos, Q, same=True)
        F[ni:] -= Q[:, None] * ggg
    F *= p.coulomb_k
    return F[:ni], F[ni:]


# ---------------------------------------------------------------- quadratic form in Q (Eqs. (5), (18), (19))


def electrode_matrix(p, ele_pos, modes=None, chunk=8192):
    """Eq. (18): A_ij (with the 4 pi/V slab reading), times coulomb_k.

    The Fourier sum sum_k w_k cos(k.(R_i - R_j)) is written with the angle
    difference identity as C diag(w) C^T + S diag(w) S^T, C = cos(k.R), S = sin(k.R).
    """
    ele_pos = np.asarray(ele_pos, dtype=np.float64).reshape(-1, 3)
    n = len(ele_pos)
    modes = enumerate_modes(p) if modes is None else modes
    kv = kvectors(p, modes)
    w = ewald_weight(p, np.sum(kv ** 2, axis=1))
    A = np.zeros((n, n))
    for s in range(0, len(kv), chunk):
        ph = ele_pos @ kv[s:s + chunk].T
        c = np.cos(ph)
        sn = np.sin(ph)
        ws = w[s:s + chunk]
        A += (c * ws) @ c.T + (sn * ws) @ sn.T
    # real space: sum over images n (excluding i=j, n=0) of the Gaussian-Gaussian kernel
    K, _ = KERNELS["gg"]
    pos = wrap_xy(p, ele_pos)
    for sh in image_shifts(p):
        d = pos[:, None, :] - pos[None, :, :] - sh[None, None, :]
        r = np.sqrt(np.sum(d * d, axis=2))
        mask = r < p.rc
        if not np.any(sh):
            np.fill_diagonal(mask, False)
        A += np.where(mask, K(p, np.where(mask, r, 1.0)), 0.0)
    cg, _ = self_constants(p)
    A += 2.0 * cg * np.eye(n)
    if p.slab:
        Z = ele_pos[:, 2]
        A += (4.0 * np.pi / p.V) * np.outer(Z, Z)
    return p.coulomb_k * A


def electrode_vector(p, ion_pos, ion_q, ele_pos, modes=None):
    """Eq. (19) without the +Delta psi entry and with the minus-sign slab reading.

    b_j = -sum_k w_k Re(exp(-i k.R_j) S1(k)) - (4 pi/V) Z_j sum q_i z_i
          - sum_i sum_n q_i [erfc(alpha r) - erfc(r/eta)]/r, times coulomb_k.
    """
    ion_pos = np.asarray(ion_pos, dtype=np.float64).reshape(-1, 3)
    ele_pos = np.asarray(ele_pos, dtype=np.float64).reshape(-1, 3)
    ion_q = np.asarray(ion_q, dtype=np.float64)
    modes = enumerate_modes(p) if modes is None else modes
    S1 = structure_factor(p, modes, ion_pos, ion_q)
    k2 = np.sum(kvectors(p, modes) ** 2, axis=1)
    bF = -fourier_potential(p, modes, ewald_weight(p, k2) * S1, ele_pos)
    bS = -(4.0 * np.pi / p.V) * ele_pos[:, 2] * (ion_q @ ion_pos[:, 2]) if p.slab else 0.0
    phi, _ = real_space(p, "ig", ele_pos, ion_pos, ion_q) if len(ion_pos) else (np.zeros(len(ele_pos)), None)
    return p.coulomb_k * (bF + bS - phi)


def constant_term(p, ion_pos, ion_q, modes=None):
    """c of Eq. (5): the Q-independent part of U_c (ion-ion real, Fourier, self, slab), times coulomb_k."""
    ion_pos = np.asarray(ion_pos, dtype=np.float64).reshape(-1, 3)
    ion_q = np.asarray(ion_q, dtype=np.float64)
    e = energy(p, ion_pos, ion_q, np.zeros((0, 3)), np.zeros(0), modes=modes)
    return e["total"]
