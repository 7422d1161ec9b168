"""Electrostatic virial (pressure) tensor of the Ewald and SRBE energies (oracle, FP64).

Test infrastructure only (see the package docstring).

The pressure tensor of an MD system is P = (sum_i m_i v_i v_i^T + W) / V, where the
virial W = -dU/d(epsilon) is the derivative of the potential energy under an affine
strain r -> (I + epsilon) r of every position and of the box, taken at epsilon = 0
with the charges held fixed.  The paper gives forces (Eqs. (21), (25)) but no
virial; this module is the reading used for the electrostatic part (the kinetic
term and any short-range force field are the caller's):

* Fourier part (Eq. (16)).  Fractional coordinates, hence S(k), do not change under
  the strain; k -> (I + epsilon)^-T k and V -> det(I + epsilon) V.  Each mode of
  U_F = 1/2 sum_k w(k) |S(k)|^2, w = 4 pi exp(-k^2/(4 alpha^2)) / (V k^2), then gives
      W_F = sum_k 1/2 w(k) |S(k)|^2 [I - 2 (1 + k^2/(4 alpha^2)) k k^T / k^2],
  summed over the charges of every kind (S = S1 + S2, ions and electrode Gaussians).
* Real part (Eq. (13)).  Every pair vector within rc (minimum image) stretches with
  the strain and the kernels (alpha, the Gaussian width eta) do not:
      W_N = -sum_pairs q_a q_b K'(r) r r^T / r,
  over ion-ion, ion-Gaussian and Gaussian-Gaussian pairs, each pair once.
* Slab term (Eq. (17)), (2 pi / V) M_z^2 with M_z = sum q z + sum Q Z: an x or y
  stretch changes V only, a z stretch V and M_z, so
      W_slab = (2 pi / V) M_z^2 diag(1, 1, -1);
  its shear components are taken as zero (the term involves only the z dipole).
* Self terms: constant, no virial.

The SRBE estimate W* replaces the Fourier sum by the estimator of Eq. (24) with the
same deterministic modes and sample as the forces (weights 4 pi exp(-k^2/4 alpha^2)
/(V k^2) on I, (G/P) 4 pi/(V k^2) per sampled mode); the bracket is unchanged, so the
estimate is unbiased for W_F.  Components are returned as [xx, yy, zz, xy, xz, yz],
times coulomb_k.
"""

import numpy as np

from . import ewald, srbe

COMPONENTS = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))


def _six(T):
    return np.array([T[a, b] for a, b in COMPONENTS])


def fourier_virial(p, m, w, S):
    """sum_k 1/2 w_k |S_k|^2 [I - 2 (1 + k^2/(4 alpha^2)) k k^T / k^2] (3 x 3, no coulomb_k)."""
    kv = ewald.kvectors(p, m)
    k2 = np.sum(kv * kv, axis=1)
    e = 0.5 * np.asarray(w) * np.abs(S) ** 2
    f = 2.0 * (1.0 + k2 / (4.0 * p.alpha ** 2)) / k2
    return np.sum(e) * np.eye(3) - np.einsum("k,ka,kb->ab", e * f, kv, kv)


def _pair_virial(p, kind, a_pos, a_q, b_pos, b_q, same):
    """-sum over pairs (a, b) within rc of q_a q_b K'(r) r r^T / r (each pair once)."""
    _, dK = ewald.KERNELS[kind]
    a_pos = ewald.wrap_xy(p, a_pos)
    b_pos = ewald.wrap_xy(p, b_pos)
    W = np.zeros((3, 3))
    for i in range(len(a_pos)):
        d = a_pos[i][None, :] - b_pos
        d[:, 0] -= p.Lx * np.round(d[:, 0] / p.Lx)
        d[:, 1] -= p.Ly * np.round(d[:, 1] / p.Ly)
        r = np.sqrt(np.sum(d * d, axis=1))
        mask = r < p.rc
        if same:
            mask[: i + 1] = False  # each pair once, no self pair
        if not np.any(mask):
            continue
        dd, rr = d[mask], r[mask]
        c = -a_q[i] * b_q[mask] * dK(p, rr) / rr
        W += np.einsum("k,ka,kb->ab", c, dd, dd)
    return W


def real_virial(p, ion_pos, ion_q, ele_pos, Q):
    """W_N over ion-ion, ion-Gaussian and Gaussian-Gaussian pairs (3 x 3, no coulomb_k)."""
    ion_pos = np.asarray(ion_pos, dtype=np.float64).reshape(-1, 3)
    ele_pos = np.asarray(ele_pos, dtype=np.float64).reshape(-1, 3)
    W = np.zeros((3, 3))
    if len(ion_pos):
        W += _pair_virial(p, "ii", ion_pos, ion_q, ion_pos, ion_q, True)
    if len(ion_pos) and len(ele_pos):
        W += _pair_virial(p, "ig", ion_pos, ion_q, ele_pos, Q, False)
    if len(ele_pos):
        W += _pair_virial(p, "gg", ele_pos, Q, ele_pos, Q, True)
    return W


def slab_virial(p, ion_pos, ion_q, ele_pos, Q):
    if not p.slab:
        return np.zeros((3, 3))
    Mz = np.asarray(ion_q) @ np.asarray(ion_pos).reshape(-1, 3)[:, 2]
    if len(Q):
        Mz += np.asarray(Q) @ np.asarray(ele_pos).reshape(-1, 3)[:, 2]
    return (2.0 * np.pi / p.V) * Mz ** 2 * np.diag([1.0, 1.0, -1.0])


def complete_virial(p, ion_pos, ion_q, ele_pos, Q, modes=None):
    """The virial of the complete energy U_c at fixed charges, [xx, yy, zz, xy, xz, yz]."""
    modes = ewald.enumerate_modes(p) if modes is None else modes
    ion_pos = np.asarray(ion_pos, dtype=np.float64).reshape(-1, 3)
    ele_pos = np.asarray(ele_pos, dtype=np.float64).reshape(-1, 3)
    S = ewald.structure_factor(p, modes, ion_pos, ion_q)
    if len(ele_pos):
        S = S + ewald.structure_factor(p, modes, ele_pos, Q)
    k2 = np.sum(ewald.kvectors(p, modes) ** 2, axis=1)
    W = fourier_virial(p, modes, ewald.ewald_weight(p, k2), S)
    W += real_virial(p, ion_pos, ion_q, ele_pos, Q) + slab_virial(p, ion_pos, ion_q, ele_pos, Q)
    return p.coulomb_k * _six(W)


def srbe_virial(p, kset, ion_pos, ion_q, ele_pos, Q):
    """The SRBE estimate W* for one sample, [xx, yy, zz, xy, xz, yz]."""
    ion_pos = np.asarray(ion_pos, dtype=np.float64).reshape(-1, 3)
    ele_pos = np.asarray(ele_pos, dtype=np.float64).reshape(-1, 3)
    m, w = srbe._combined(p, kset)
    S = ewald.structure_factor(p, m, ion_pos, ion_q)
    if len(ele_pos):
        S = S + ewald.structure_factor(p, m, ele_pos, Q)
    W = fourier_virial(p, m, w, S)
    W += real_virial(p, ion_pos, ion_q, ele_pos, Q) + slab_virial(p, ion_pos, ion_q, ele_pos, Q)
    return p.coulomb_k * _six(W)
