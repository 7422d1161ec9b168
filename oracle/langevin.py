"""Euler-Maruyama step of the Langevin thermostat (oracle, FP64).

Test infrastructure only (see the package docstring).

Sec. 3 of the paper (the discrete update after the Langevin system it writes for
SRBE-driven dynamics): for every ion,

    r^{n+1} = r^n + v^n dt
    v^{n+1} = v^n + (F^n - gamma v^n) dt / m + sqrt(2 gamma / beta) dW / m,
    dW ~ N(0, dt) per component.

The confinement is a reading (the paper's force field holds the ions between the
walls; none is modelled here): x and y wrap into [0, L); z is reflected specularly
into [zlo, zhi] as often as it takes to land inside: with W = zhi - zlo,
k = floor((z - zlo) / W) reflections and t = (z - zlo) - k W, z becomes zlo + t for
even k and zhi - t for odd k (then clamped into [zlo, zhi] against rounding), and
v_z changes sign once per reflection.  One reflection is z -> 2 zlo - z below or
2 zhi - z above.  A z already inside is left unchanged.

Normal deviates: Philox4x64-10 with key (seed, 1) and counter (ion index, step, 3, 0);
the four words map to uniforms in (0, 1) by ((w >> 12) + 1/2) 2^-52, and Box-Muller
gives z_x = sqrt(-2 ln U0) cos(2 pi U1), z_y = sqrt(-2 ln U0) sin(2 pi U1),
z_z = sqrt(-2 ln U2) cos(2 pi U3); dW = sqrt(dt) z.
"""

import numpy as np

from . import philox

PURPOSE_LANGEVIN = 3


def normals(seed, step, n):
    """(n, 3) standard normal deviates of the update (counter layout in the module docstring)."""
    idx = np.arange(n, dtype=np.uint64)
    ctr = np.stack([idx, np.full(n, step, dtype=np.uint64), np.full(n, PURPOSE_LANGEVIN, dtype=np.uint64),
                    np.zeros(n, dtype=np.uint64)], axis=1)
    w = philox.philox4x64_10(ctr, np.array([seed, 1], dtype=np.uint64))
    U = philox.u01_open(w)
    r0 = np.sqrt(-2.0 * np.log(U[:, 0]))
    r2 = np.sqrt(-2.0 * np.log(U[:, 2]))
    return np.stack([r0 * np.cos(2.0 * np.pi * U[:, 1]), r0 * np.sin(2.0 * np.pi * U[:, 1]),
                     r2 * np.cos(2.0 * np.pi * U[:, 3])], axis=1)


def euler_maruyama(pos, vel, F, mass, gamma, beta, dt, Lx, Ly, zlo, zhi, seed, step, symplectic=False):
    """One update; pos, vel, F (n, 3), mass (n,).  Returns (pos, vel) after the step.

    symplectic: move the positions with the updated velocity, r + v^{n+1} dt (the
    symplectic Euler ordering of the same update, a reading for the dynamics: the
    printed r + v^n dt gains energy on every stiff oscillation, by 1 + (omega dt)^2 per
    step, which outruns the friction on steep contacts).
    """
    pos = np.asarray(pos, dtype=np.float64)
    vel = np.asarray(vel, dtype=np.float64)
    F = np.asarray(F, dtype=np.float64)
    m = np.asarray(mass, dtype=np.float64)[:, None]
    dW = np.sqrt(dt) * normals(seed, step, len(pos))
    v = vel + (F - gamma * vel) * dt / m + np.sqrt(2.0 * gamma / beta) * dW / m
    r = pos + (v if symplectic else vel) * dt
    r[:, 0] = np.mod(r[:, 0], Lx)
    r[:, 1] = np.mod(r[:, 1], Ly)
    out = (r[:, 2] < zlo) | (r[:, 2] > zhi)
    W = zhi - zlo
    k = np.floor((r[out, 2] - zlo) / W)
    t = np.clip((r[out, 2] - zlo) - k * W, 0.0, W)
    odd = np.fmod(k, 2.0) != 0.0
    r[out, 2] = np.clip(np.where(odd, zhi - t, zlo + t), zlo, zhi)
    v[out, 2] *= np.where(odd, -1.0, 1.0)
    return r, v
