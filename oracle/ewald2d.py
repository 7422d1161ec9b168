"""Exact quasi-2D Ewald sum and brute-force 2-D image sums (oracle pins only).

Test infrastructure only (see the package docstring).

Eq. (14) integrates over k_z instead of summing the zero-padded lattice of
Eq. (16); for point charges the integral has a closed form (the Ewald2D sum the
paper cites for the quasi-2D problem).  With A = Lx Ly, rho_ij the in-plane and
z_ij the normal separation:

  int dk_z cos(k_z z) exp(-k_z^2/(4 alpha^2)) / (kd^2 + k_z^2)
      = pi/(2 kd) exp(kd^2/(4 alpha^2)) [exp(kd z) erfc(kd/(2 alpha) + alpha z)
                                        + exp(-kd z) erfc(kd/(2 alpha) - alpha z)]

for an in-plane wave number kd > 0, and for kd = 0 (neutral systems, the
divergent constant cancels) the regularised integral is
-pi [z erf(alpha z) + exp(-alpha^2 z^2)/(alpha sqrt(pi))].  Eq. (14) then gives

  U_F^Q2D = pi/(2A) sum_{kd != 0} 1/kd sum_ij q_i q_j cos(kd.rho_ij) [ ... ]
            - pi/A sum_ij q_i q_j [z_ij erf(alpha z_ij) + exp(-alpha^2 z_ij^2)/(alpha sqrt(pi))].

U_c = U_N (2-D images) + U_F^Q2D - alpha/sqrt(pi) sum q^2.  Only point charges
(ions) are handled; the EW3DC energy of ``oracle.ewald`` must approach this as
lambda grows (Sec. 2, the zero-padding discussion after Eq. (17)).
"""

import numpy as np
from scipy.special import erfc, erf, erfcx

from . import ewald


def _exp_erfc(s, x):
    """exp(s) erfc(x), evaluated as exp(s - x^2) erfcx(x) where x > 0 so that neither factor overflows."""
    pos = x > 0
    xs = np.where(pos, x, 0.0)
    a = np.exp(np.where(pos, s - xs * xs, 0.0)) * erfcx(xs)
    b = np.exp(np.where(pos, 0.0, s)) * erfc(np.where(pos, 0.0, x))
    return np.where(pos, a, b)


def energy_q2d(p, pos, q, kd_tol=1e-16):
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    q = np.asarray(q, dtype=np.float64)
    A = p.Lx * p.Ly
    a = p.alpha
    # in-plane modes with exp(-kd^2/(4 alpha^2)) >= kd_tol; the z-factor erfc(.)<=2 bounds the rest
    k2max = 4.0 * a * a * np.log(1.0 / kd_tol)
    mx_max = int(np.floor(np.sqrt(k2max) * p.Lx / (2 * np.pi)))
    my_max = int(np.floor(np.sqrt(k2max) * p.Ly / (2 * np.pi)))
    dx = pos[:, None, :] - pos[None, :, :]
    qq = q[:, None] * q[None, :]
    z = dx[:, :, 2]
    u = 0.0
    for mx in range(-mx_max, mx_max + 1):
        for my in range(-my_max, my_max + 1):
            if mx == 0 and my == 0:
                continue
            kx = 2 * np.pi * mx / p.Lx
            ky = 2 * np.pi * my / p.Ly
            kd = np.hypot(kx, ky)
            if kd * kd > k2max:
                continue
            c = np.cos(kx * dx[:, :, 0] + ky * dx[:, :, 1])
            t1 = _exp_erfc(kd * z, kd / (2 * a) + a * z)
            t2 = _exp_erfc(-kd * z, kd / (2 * a) - a * z)
            u += (np.pi / (2 * A)) / kd * np.sum(qq * c * (t1 + t2))
    u0 = -(np.pi / A) * np.sum(qq * (z * erf(a * z) + np.exp(-(a * z) ** 2) / (a * np.sqrt(np.pi))))
    # The 1/(4 pi A) prefactor of Eq. (14) times 4 pi leaves 1/A, which the two sums carry.
    u_f = u + u0
    phi, _ = ewald.real_space(p, "ii", pos, pos, q, same=True)
    u_n = 0.5 * q @ phi
    u_self = -(a / np.sqrt(np.pi)) * np.sum(q * q)
    return p.coulomb_k * (u_n + u_f + u_self)


def energy_images(p, pos, q, R, width=None):
    """Disc summation of the total Coulomb energy over 2-D images, |n o l| < R.

    1/2 sum_ij sum_n' q_i q_j phi_ij(|r_ij + n o l|) with phi_ij = erf(r/s_ij)/r,
    s_ij^2 = w_i^2 + w_j^2 (w = 0 for a point charge, eta for the Gaussian of
    Eq. (1); two Gaussians of widths w_i, w_j interact as one of width s_ij), plus
    the self energy Q^2/(sqrt(2 pi) eta) of every Gaussian.  Returns coulomb_k times
    the sum; the caller adds the analytic dipole tail (``disc_tail``).
    """
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    q = np.asarray(q, dtype=np.float64)
    w = np.zeros(len(q)) if width is None else np.asarray(width, dtype=np.float64)
    s = np.sqrt(w[:, None] ** 2 + w[None, :] ** 2)
    nx = int(np.ceil(R / p.Lx))
    ny = int(np.ceil(R / p.Ly))
    d = pos[:, None, :] - pos[None, :, :]
    qq = q[:, None] * q[None, :]
    u = 0.0
    for ix in range(-nx, nx + 1):
        for iy in range(-ny, ny + 1):
            sx, sy = ix * p.Lx, iy * p.Ly
            if np.hypot(sx, sy) >= R:
                continue
            r = np.sqrt((d[:, :, 0] + sx) ** 2 + (d[:, :, 1] + sy) ** 2 + d[:, :, 2] ** 2)
            if ix == 0 and iy == 0:
                np.fill_diagonal(r, np.inf)
            ker = np.where(s > 0, erf(r / np.where(s > 0, s, 1.0)), 1.0) / r
            u += 0.5 * np.sum(qq * ker)
    g = w > 0
    u += np.sum(q[g] ** 2 / (np.sqrt(2.0 * np.pi) * w[g]))
    return p.coulomb_k * u


def disc_tail(p, pos, q, R):
    """Energy of the images beyond the disc |n o l| >= R, to leading order.

    For a neutral cell with dipole moment m the far images interact as dipoles;
    averaging (m.m - 3 (m.n^)^2)/rho^3 over in-plane directions and integrating
    2 pi rho drho / (Lx Ly) from R to infinity gives (pi/(Lx Ly R)) (m_z^2 - |m_xy|^2/2).
    """
    m = np.asarray(q, dtype=np.float64) @ np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    return p.coulomb_k * (np.pi / (p.Lx * p.Ly * R)) * (m[2] ** 2 - 0.5 * (m[0] ** 2 + m[1] ** 2))
