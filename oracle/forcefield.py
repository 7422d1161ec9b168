"""Short-range force field for SRBE-driven dynamics (oracle, FP64).

Test infrastructure only (see the package docstring).

The paper runs its dynamics (Sec. 4) with a coarse-grained force field it does not
give.  This stand-in is a reading: it only has to keep ions apart, keep them between
the walls and hold a molecule's sites together, so that the Langevin dynamics of Sec. 3
driven by the SRBE forces can run and show the electrodes charging.  Its terms:

* WCA repulsion between sites of different molecules,
      U(r) = 4 eps [(s/r)^12 - (s/r)^6] + eps   for r < 2^(1/6) s, else 0;
* a 9-3 wall at z = zlo (acting on sites above it) and one at z = zhi (below it),
  cut and shifted at its minimum so that it only repels:
      U(d) = eps_w [(2/15)(s_w/d)^9 - (s_w/d)^3] - U_min   for d < d_min = (2/5)^(1/6) s_w,
      d = z - zlo or zhi - z;
* harmonic bonds between listed pairs of sites, U = (k/2)(r - r0)^2.

Distances use the minimum image in x and y.  Every function here is the definition
written out over all pairs (O(N^2)): for the small systems of the tests.
"""

import numpy as np


def wca(eps, sigma, r):
    """WCA energy and dU/dr at distances r (zero beyond 2^(1/6) sigma)."""
    r = np.asarray(r, dtype=np.float64)
    rc = 2.0 ** (1.0 / 6.0) * sigma
    inside = r < rc
    sr6 = np.where(inside, (sigma / np.where(inside, r, 1.0)) ** 6, 0.0)
    u = np.where(inside, 4.0 * eps * (sr6 * sr6 - sr6) + eps, 0.0)
    du = np.where(inside, -24.0 * eps * (2.0 * sr6 * sr6 - sr6) / np.where(inside, r, 1.0), 0.0)
    return u, du


def wall93(eps, sigma, d):
    """Repulsive 9-3 wall energy and dU/dd at distances d from the wall plane."""
    d = np.asarray(d, dtype=np.float64)
    dmin = (2.0 / 5.0) ** (1.0 / 6.0) * sigma
    umin = eps * ((2.0 / 15.0) * (sigma / dmin) ** 9 - (sigma / dmin) ** 3)
    inside = d < dmin
    dd = np.where(inside, d, 1.0)
    u = np.where(inside, eps * ((2.0 / 15.0) * (sigma / dd) ** 9 - (sigma / dd) ** 3) - umin, 0.0)
    du = np.where(inside, eps * (-(18.0 / 15.0) * sigma ** 9 / dd ** 10 + 3.0 * sigma ** 3 / dd ** 4), 0.0)
    return u, du


def _pair_vectors(pos, Lx, Ly):
    d = pos[:, None, :] - pos[None, :, :]
    d[..., 0] -= Lx * np.round(d[..., 0] / Lx)
    d[..., 1] -= Ly * np.round(d[..., 1] / Ly)
    return d


def energy(pos, mol, bonds, ff, Lx, Ly):
    """Total short-range energy.  pos (N, 3); mol (N,) molecule index; bonds: (i, j, r0) triples;
    ff: dict with wca_eps, wca_sigma, wall_eps, wall_sigma, wall_zlo, wall_zhi, bond_k."""
    pos = np.asarray(pos, dtype=np.float64)
    mol = np.asarray(mol)
    d = _pair_vectors(pos, Lx, Ly)
    r = np.sqrt(np.sum(d * d, axis=2))
    iu = np.triu_indices(len(pos), 1)
    other = mol[iu[0]] != mol[iu[1]]
    u_pair, _ = wca(ff["wca_eps"], ff["wca_sigma"], r[iu][other])
    u_lo, _ = wall93(ff["wall_eps"], ff["wall_sigma"], pos[:, 2] - ff["wall_zlo"])
    u_hi, _ = wall93(ff["wall_eps"], ff["wall_sigma"], ff["wall_zhi"] - pos[:, 2])
    u_bond = 0.0
    for i, j, r0 in bonds:
        rij = np.sqrt(np.sum(d[i, j] ** 2))
        u_bond += 0.5 * ff["bond_k"] * (rij - r0) ** 2
    return float(np.sum(u_pair) + np.sum(u_lo) + np.sum(u_hi) + u_bond)


def forces(pos, mol, bonds, ff, Lx, Ly):
    """-grad of ``energy`` with respect to every site (N, 3)."""
    pos = np.asarray(pos, dtype=np.float64)
    mol = np.asarray(mol)
    n = len(pos)
    d = _pair_vectors(pos, Lx, Ly)
    r = np.sqrt(np.sum(d * d, axis=2))
    np.fill_diagonal(r, 1.0)
    _, du = wca(ff["wca_eps"], ff["wca_sigma"], r)
    du[mol[:, None] == mol[None, :]] = 0.0
    np.fill_diagonal(du, 0.0)
    F = -np.einsum("ij,ijk->ik", du / r, d)
    _, dlo = wall93(ff["wall_eps"], ff["wall_sigma"], pos[:, 2] - ff["wall_zlo"])
    _, dhi = wall93(ff["wall_eps"], ff["wall_sigma"], ff["wall_zhi"] - pos[:, 2])
    F[:, 2] += -dlo + dhi
    for i, j, r0 in bonds:
        rij = np.sqrt(np.sum(d[i, j] ** 2))
        f = -ff["bond_k"] * (rij - r0) * d[i, j] / rij  # on i
        F[i] += f
        F[j] -= f
    return F
