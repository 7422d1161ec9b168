"""Metropolis sampler of the random batch (oracle, FP64).

Test infrastructure only (see the package docstring).

Sec. 3, Eqs. (26)-(29).  Target: P(k) = exp(-k^2/(4 alpha^2)) / G on L_k \\ I.
Proposal: per axis u_d ~ N(0, sigma_d^2), m*_d = round(u_d); its probability mass
is q_d(m) = int_{m-1/2}^{m+1/2} sqrt(pi/(alpha^2 L_d^2)) exp(-pi^2 x^2/(alpha L_d)^2) dx
(Eq. (28)).  A proposal outside L_k \\ I (the origin or a mode of I) has target
probability zero and is rejected; otherwise it is accepted with probability
min{1, P(k*) q(m) / (P(k) q(m*))} (Eq. (29)), where q(m) = prod_d q_d(m_d).

Readings:
* Proposal variance.  The text gives alpha^2 L_d^2/(2 pi)^2, but the density in
  Eq. (28) is a Gaussian of variance alpha^2 L_d^2/(2 pi^2); only with the latter is
  q_d the probability of round(u_d), which Eq. (29) needs for the chain to target
  P(k).  We draw u_d with sigma_d = alpha L_d/(sqrt(2) pi).
* Chain start and length (not stated).  A fresh chain per (seed, stream, step):
  its initial state is the first proposal inside L_k \\ I from a separate start
  sequence (at most 64 tries; if all 64 fail, the mode (1, 0, 0)); then P
  Metropolis iterations, each contributing its current state (a rejection repeats
  the state).  Duplicates count with multiplicity.
* A proposal y in L_k \\ I is accepted when d = log r(y) - log r(x) >= 0 or
  log U < d, the logarithm of U < min{1, r(y)/r(x)} with r the ratio of Eq. (29).
* Rounding is round-half-up, m = floor(u + 1/2).

Random numbers: Philox4x64-10 (``oracle.philox``) with key (seed, stream) and
counter (index, step, purpose, 0); purpose 0 = proposal of iteration index,
1 = acceptance uniform of iteration index, 2 = start-sequence proposal index.
A proposal block's four words w0..w3 give uniforms U_i = ((w_i >> 12) + 1/2) 2^-52
and normals by Box-Muller: z_x = sqrt(-2 ln U0) cos(2 pi U1),
z_y = sqrt(-2 ln U0) sin(2 pi U1), z_z = sqrt(-2 ln U2) cos(2 pi U3).
The acceptance uniform is U from word 0 of its block.
"""

import numpy as np
from scipy.special import erfc

from . import philox

PURPOSE_PROPOSAL = 0
PURPOSE_ACCEPT = 1
PURPOSE_START = 2
PURPOSE_IID_PROPOSAL = 3
PURPOSE_IID_ACCEPT = 4
START_TRIES = 64
IID_MAX_ATTEMPTS = 65536


def proposal_sigma(p):
    """sigma_d = alpha L_d / (sqrt(2) pi) per axis (reading above)."""
    return p.alpha * p.L / (np.sqrt(2.0) * np.pi)


def q_axis(m, alpha, L):
    """Eq. (28): probability that round(u) = m for u of density sqrt(pi/(alpha^2 L^2)) exp(-pi^2 x^2/(alpha L)^2).

    Written with erfc on |m| so that tails do not cancel:
    q(m) = 1/2 [erfc(c (|m| - 1/2)) - erfc(c (|m| + 1/2))], c = pi/(alpha L).
    """
    a = np.abs(np.asarray(m, dtype=np.float64))
    c = np.pi / (alpha * L)
    return 0.5 * (erfc(c * (a - 0.5)) - erfc(c * (a + 0.5)))


def log_ratio(p, m):
    """log[ exp(-k^2/(4 alpha^2)) / prod_d q_d(m_d) ], the importance ratio of Eq. (29)."""
    m = np.asarray(m, dtype=np.float64).reshape(-1, 3)
    k2 = np.sum((2.0 * np.pi * m / p.L) ** 2, axis=1)
    lq = (np.log(q_axis(m[:, 0], p.alpha, p.Lx)) + np.log(q_axis(m[:, 1], p.alpha, p.Ly))
          + np.log(q_axis(m[:, 2], p.alpha, p.Lz)))
    return -k2 / (4.0 * p.alpha ** 2) - lq


def valid(p, m):
    """True where m lies in L_k \\ I (not the origin, not a deterministic mode)."""
    m = np.asarray(m).reshape(-1, 3)
    inplane0 = (m[:, 0] == 0) & (m[:, 1] == 0)
    return ~(inplane0 & (np.abs(m[:, 2]) <= p.M))


def _blocks(seed, stream, step, purpose, idx):
    idx = np.asarray(idx, dtype=np.uint64)
    ctr = np.zeros((len(idx), 4), dtype=np.uint64)
    ctr[:, 0] = idx
    ctr[:, 1] = np.uint64(step)
    ctr[:, 2] = np.uint64(purpose)
    key = np.array([seed, stream], dtype=np.uint64)
    return philox.philox4x64_10(ctr, key)


def proposals(p, seed, stream, step, purpose, idx):
    """Rounded Gaussian proposals (int64 (n, 3)) for the given counter indices."""
    w = _blocks(seed, stream, step, purpose, idx)
    U = philox.u01_open(w)
    r0 = np.sqrt(-2.0 * np.log(U[:, 0]))
    r2 = np.sqrt(-2.0 * np.log(U[:, 2]))
    z = np.stack([r0 * np.cos(2.0 * np.pi * U[:, 1]),
                  r0 * np.sin(2.0 * np.pi * U[:, 1]),
                  r2 * np.cos(2.0 * np.pi * U[:, 3])], axis=1)
    u = proposal_sigma(p)[None, :] * z
    return np.floor(u + 0.5).astype(np.int64)


def acceptance_uniforms(seed, stream, step, idx):
    w = _blocks(seed, stream, step, PURPOSE_ACCEPT, idx)
    return philox.u01_open(w[:, 0])


def draw_kset(p, seed, stream, step, P=None):
    """Draw one batch of P modes (int64 (P, 3)) with the chain described above.

    Returns (kset, n_accepted).
    """
    P = p.P if P is None else P
    start = proposals(p, seed, stream, step, PURPOSE_START, np.arange(START_TRIES))
    ok = np.nonzero(valid(p, start))[0]
    x = start[ok[0]].copy() if len(ok) else np.array([1, 0, 0], dtype=np.int64)
    if P == 0:
        return np.zeros((0, 3), dtype=np.int64), 0
    y = proposals(p, seed, stream, step, PURPOSE_PROPOSAL, np.arange(P))
    U = acceptance_uniforms(seed, stream, step, np.arange(P))
    ly = log_ratio(p, y)
    vy = valid(p, y)
    lx = float(log_ratio(p, x)[0])
    out = np.zeros((P, 3), dtype=np.int64)
    nacc = 0
    lU = np.log(U)
    for l in range(P):
        if vy[l]:
            d = ly[l] - lx
            if d >= 0.0 or lU[l] < d:
                x = y[l]
                lx = float(ly[l])
                nacc += 1
        out[l] = x
    return out, nacc


def iid_draw_kset(p, seed, stream, step, P=None):
    """P independent draws from the same target by rejection sampling (the i.i.d. option).

    Attempt a draws its proposal m = round(sigma z) exactly as above from counter
    (a, step, 3, 0) and its uniform U from word 0 of counter (a, step, 4, 0).  Per axis
    exp(-m^2/(2 sigma_d^2)) / q_d(m) is largest at m = 0 (q_d(m) is the target's density
    integrated over [m - 1/2, m + 1/2], which shrinks more slowly than the density as |m|
    grows), so r(m) <= r(0) with r the ratio of Eq. (29), and accepting a proposal in
    L_k \\ I when log U < log r(m) - log r(0) gives exact draws from the target.  The
    sample is the accepted proposals in attempt order.  After IID_MAX_ATTEMPTS attempts
    the rest of the sample is (1, 0, 0) (reachable only when the bound is loose, e.g.
    with most of the proposal's mass on I).

    Returns (kset, attempts): attempts = the index of the attempt that completed the
    sample, plus one (IID_MAX_ATTEMPTS if it was not completed).
    """
    P = p.P if P is None else P
    out = np.zeros((P, 3), dtype=np.int64)
    if P == 0:
        return out, 0
    l0 = float(log_ratio(p, np.zeros((1, 3)))[0])
    filled = 0
    chunk = 1024
    for a0 in range(0, IID_MAX_ATTEMPTS, chunk):
        idx = np.arange(a0, a0 + chunk)
        y = proposals(p, seed, stream, step, PURPOSE_IID_PROPOSAL, idx)
        w = _blocks(seed, stream, step, PURPOSE_IID_ACCEPT, idx)
        lU = np.log(philox.u01_open(w[:, 0]))
        ok = valid(p, y)
        ok[ok] = lU[ok] < log_ratio(p, y[ok]) - l0
        for a in np.nonzero(ok)[0]:
            out[filled] = y[a]
            filled += 1
            if filled == P:
                return out, a0 + int(a) + 1
    out[filled:] = (1, 0, 0)
    return out, IID_MAX_ATTEMPTS
