"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test compares the oracle with something other than itself: a library
routine, a closed form, a brute-force sum, a derivative taken numerically, or an
identity the paper states.  A dropped term, a wrong sign or factor, or a
transposed operand in the oracle fails at least one of them.
"""

import numpy as np
import pytest
from scipy.stats import norm

from oracle import cp, ewald, ewald2d, langevin, philox, sampler, srbe


# ---------------------------------------------------------------- helpers


def tiny_system(seed=5, n_ion=6, lam=3.0, alpha=5.0, M=4, P=20, tol=1e-14):
    """Two 3x3 Gaussian walls and a few ions (cheap enough for finite differences)."""
    rng = np.random.default_rng(seed)
    Lx, Ly, H = 1.2, 1.2, 2.0
    g = (np.arange(3) + 0.5) * 0.4
    X, Y = np.meshgrid(g, g, indexing="ij")
    wall = np.column_stack([X.ravel(), Y.ravel()])
    ele = np.vstack([np.column_stack([wall, np.zeros(9)]), np.column_stack([wall, np.full(9, H)])])
    side = np.array([-1] * 9 + [1] * 9)
    ion = np.column_stack([rng.uniform(0, Lx, n_ion), rng.uniform(0, Ly, n_ion),
                           rng.uniform(0.4, H - 0.4, n_ion)])
    q = np.resize([0.8, -0.8], n_ion).astype(float)
    p = ewald.Params(Lx=Lx, Ly=Ly, H=H, lam=lam, alpha=alpha, eta=0.08, rc=0.6, coulomb_k=1.44,
                     M=M, P=P, kspace_tol=tol)
    return p, ion, q, ele, side


# ---------------------------------------------------------------- Philox


def test_philox_matches_numpy_reference():
    # numpy's Philox bit generator is Philox4x64-10; it increments its counter
    # before each block, so counter c with numpy gives our block c + 1.
    rng = np.random.default_rng(0)
    for _ in range(20):
        key = rng.integers(0, 2 ** 63, size=2, dtype=np.uint64)
        c = rng.integers(0, 2 ** 63, size=4, dtype=np.uint64)
        ref = np.random.Philox(counter=c, key=key).random_raw(4)
        c1 = c.copy()
        c1[0] += np.uint64(1)
        assert np.array_equal(philox.philox4x64_10(c1, key), ref)
    # carry out of the low counter word
    key = np.array([7, 9], dtype=np.uint64)
    ref = np.random.Philox(counter=np.array([2 ** 64 - 1, 5, 0, 0], dtype=np.uint64), key=key).random_raw(4)
    assert np.array_equal(philox.philox4x64_10(np.array([0, 6, 0, 0], dtype=np.uint64), key), ref)


def test_uniforms_open_interval():
    u = philox.u01_open(np.array([0, 2 ** 64 - 1], dtype=np.uint64))
    assert 0.0 < u[0] < 1e-15 and 1.0 - 1e-15 < u[1] < 1.0
    assert u[0] == 2.0 ** -53 and u[1] == 1.0 - 2.0 ** -53


# ---------------------------------------------------------------- G and the proposal


def test_G_equals_bruteforce_sum():
    p = ewald.Params(Lx=2.4, Ly=2.4, H=8.0, lam=3.0, alpha=3.0, M=10)
    m = ewald.enumerate_modes(p, tol=1e-300)
    k2 = np.sum(ewald.kvectors(p, m) ** 2, axis=1)
    inI = (m[:, 0] == 0) & (m[:, 1] == 0) & (np.abs(m[:, 2]) <= p.M)
    brute = np.sum(np.exp(-k2[~inI] / (4 * p.alpha ** 2)))
    assert srbe.normaliser_G(p) == pytest.approx(brute, rel=1e-12)
    assert srbe.normaliser_G(p) == pytest.approx(650.6838622, rel=1e-8)


def test_q_axis_is_pmf_of_rounded_gaussian():
    # Eq. (28) with the proposal variance alpha^2 L^2/(2 pi^2): q_d(m) must be the
    # probability that round(u) = m for u ~ N(0, sigma^2) (library normal CDF).
    for alpha, L in [(3.0, 2.4), (3.5, 36.0), (3.0, 300.0)]:
        sig = alpha * L / (np.sqrt(2) * np.pi)
        m = np.arange(-int(9 * sig) - 3, int(9 * sig) + 4)
        ref = norm.cdf((m + 0.5) / sig) - norm.cdf((m - 0.5) / sig)
        got = sampler.q_axis(m, alpha, L)
        assert np.max(np.abs(got - ref)) < 1e-14
        assert abs(np.sum(got) - 1.0) < 1e-12


def test_sampler_distribution_chi2():
    # Frequencies of sampled modes against P(k) = exp(-k^2/4a^2)/G on L_k \ I.
    # Chains are thinned (every 10th state; acceptance ~0.8, so states 10 apart
    # are independent to ~1e-7) to give independent counts.
    p = ewald.Params(Lx=1.2, Ly=1.2, H=1.5, lam=2.0, alpha=3.0, M=2)
    P, thin, chains = 200, 10, 1000
    counts = {}
    nacc = 0
    for c in range(chains):
        ks, na = sampler.draw_kset(p, seed=42, stream=c, step=3, P=P)
        assert np.all(sampler.valid(p, ks))
        nacc += na
        for row in map(tuple, ks[thin - 1::thin]):
            counts[row] = counts.get(row, 0) + 1
    n = sum(counts.values())
    assert nacc / (chains * P) > 0.75
    G = srbe.normaliser_G(p)
    allm = ewald.enumerate_modes(p, tol=1e-30)
    allm = allm[sampler.valid(p, allm)]
    pk = np.exp(-np.sum(ewald.kvectors(p, allm) ** 2, axis=1) / (4 * p.alpha ** 2)) / G
    order = np.argsort(-pk)[:40]
    obs = np.array([counts.get(tuple(allm[i]), 0) for i in order], dtype=float)
    exp = n * pk[order]
    obs = np.append(obs, n - obs.sum())
    exp = np.append(exp, n - exp.sum())
    chi2 = np.sum((obs - exp) ** 2 / exp)
    assert chi2 < 90.0  # 40 degrees of freedom: p ~ 1e-5


def test_iid_sampler_distribution_and_acceptance():
    # The i.i.d. option draws every mode exactly from P(k) = exp(-k^2/4a^2)/G on L_k \ I
    # (no chain, no thinning): chi^2 of the counts against P(k); and its acceptance is the
    # rejection sampler's exact rate, sum over L_k \ I of q(m) r(m)/r(0) = G prod_d q_d(0),
    # which the attempt counts must reproduce within 5 standard errors.
    p = ewald.Params(Lx=1.2, Ly=1.2, H=1.5, lam=2.0, alpha=3.0, M=2)
    P, draws = 200, 400
    counts = {}
    attempts = 0
    for c in range(draws):
        ks, att = sampler.iid_draw_kset(p, seed=42, stream=c, step=3, P=P)
        assert np.all(sampler.valid(p, ks))
        attempts += att
        for row in map(tuple, ks):
            counts[row] = counts.get(row, 0) + 1
    n = sum(counts.values())
    G = srbe.normaliser_G(p)
    allm = ewald.enumerate_modes(p, tol=1e-30)
    allm = allm[sampler.valid(p, allm)]
    pk = np.exp(-np.sum(ewald.kvectors(p, allm) ** 2, axis=1) / (4 * p.alpha ** 2)) / G
    order = np.argsort(-pk)[:40]
    obs = np.array([counts.get(tuple(allm[i]), 0) for i in order], dtype=float)
    exp = n * pk[order]
    obs = np.append(obs, n - obs.sum())
    exp = np.append(exp, n - exp.sum())
    chi2 = np.sum((obs - exp) ** 2 / exp)
    assert chi2 < 90.0  # 40 degrees of freedom: p ~ 1e-5
    rate = G * np.prod([sampler.q_axis(0, p.alpha, L) for L in p.L])
    assert 0.0 < rate < 1.0
    # draws of P accepted: attempts - P is negative binomial, mean P (1 - rate) / rate
    mean = draws * P / rate
    sd = np.sqrt(draws * P * (1.0 - rate)) / rate
    assert abs(attempts - mean) < 5.0 * sd, (attempts, mean, sd)


def test_sampler_never_returns_deterministic_modes():
    p = ewald.Params(Lx=3.4, Ly=3.7, H=12.0, lam=3.0, alpha=3.5, M=13)
    for step in range(5):
        ks, _ = sampler.draw_kset(p, seed=7, stream=0, step=step, P=500)
        assert np.all(sampler.valid(p, ks))


# ---------------------------------------------------------------- Ewald core


def test_nacl_madelung():
    a0 = 0.5
    pts, qs = [], []
    for i in range(4):
        for j in range(4):
            for k in range(4):
                pts.append([i * a0 / 2, j * a0 / 2, k * a0 / 2])
                qs.append((-1) ** (i + j + k))
    pts, qs = np.array(pts), np.array(qs, float)
    L = 2 * a0
    p = ewald.Params(Lx=L, Ly=L, H=L, lam=1.0, alpha=12.0, rc=0.4995 * L, coulomb_k=1.0,
                     slab=False, periodic_z=True, kspace_tol=1e-18)
    E = ewald.energy(p, pts, qs, np.zeros((0, 3)), np.zeros(0))["total"]
    madelung = 1.747564594633182
    assert E == pytest.approx(-len(qs) / 2 * madelung / (a0 / 2), rel=1e-10)


def test_alpha_independence_3d():
    rng = np.random.default_rng(2)
    L = 1.0
    pos = rng.uniform(0, L, size=(8, 3))
    q = np.array([1, -1, 0.5, -0.5, 0.3, -0.3, 1.2, -1.2])
    Es, Fs = [], []
    for alpha in (12.0, 14.0, 16.0):
        p = ewald.Params(Lx=L, Ly=L, H=L, lam=1.0, alpha=alpha, rc=0.499, coulomb_k=1.0,
                         slab=False, periodic_z=True, kspace_tol=1e-18)
        Es.append(ewald.energy(p, pos, q, np.zeros((0, 3)), np.zeros(0))["total"])
        Fs.append(ewald.forces(p, pos, q, np.zeros((0, 3)), np.zeros(0))[0])
    assert np.ptp(Es) < 1e-10 * abs(Es[0])
    assert np.max(np.abs(Fs[1] - Fs[0])) < 1e-9 * np.max(np.abs(Fs[0]))
    assert np.max(np.abs(Fs[2] - Fs[0])) < 1e-9 * np.max(np.abs(Fs[0]))


def test_de_leeuw_perram_smith_spherical_sum():
    # A 3-D periodic cell summed directly over spherical shells of image cells (in
    # vacuum) converges to the tinfoil Ewald energy plus 2 pi |M|^2 / (3 V), M the
    # cell's dipole (de Leeuw, Perram and Smith): pins the oracle's 3-D Ewald core
    # against a brute-force Coulomb sum, including its dipole dependence.
    rng = np.random.default_rng(11)
    L = 1.0
    for q in (np.array([1.0, -1.0, 0.5, -0.5]), np.array([0.7, -0.2, -0.9, 0.4, 0.3, -0.3, 0.6, -0.6])):
        pos = rng.uniform(0, L, size=(len(q), 3))
        p = ewald.Params(Lx=L, Ly=L, H=L, lam=1.0, alpha=12.0, rc=0.499, coulomb_k=1.0,
                         slab=False, periodic_z=True, kspace_tol=1e-18)
        E_ew = ewald.energy(p, pos, q, np.zeros((0, 3)), np.zeros(0))["total"]
        M = (q[:, None] * pos).sum(0)
        dipole = 2 * np.pi / (3 * L ** 3) * (M @ M)
        R = 48
        r = np.arange(-R, R + 1)
        n = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3)
        n = n[(n ** 2).sum(1) <= R * R].astype(float) * L
        d = pos[:, None, :] - pos[None, :, :]
        qq = q[:, None] * q[None, :]
        direct = 0.0
        for c in range(0, len(n), 20000):
            x = d[None] + n[c:c + 20000, None, None, :]
            rr = np.sqrt((x ** 2).sum(-1))
            with np.errstate(divide="ignore"):
                t = qq[None] / rr
            t[~np.isfinite(t)] = 0.0  # the charge itself in the home cell
            direct += 0.5 * t.sum()
        assert dipole > 1e-3 * abs(E_ew)  # the dipole term is not negligible here
        assert direct == pytest.approx(E_ew + dipole, rel=2e-8, abs=0)
        assert abs(direct - E_ew) > 0.5 * dipole


def test_ewald2d_closed_form_vs_image_sum():
    rng = np.random.default_rng(3)
    Lx, Ly, H = 1.0, 1.2, 1.5
    pos = np.column_stack([rng.uniform(0, Lx, 6), rng.uniform(0, Ly, 6), rng.uniform(0.2, H - 0.2, 6)])
    q = np.array([1, -1, 1, -1, 0.5, -0.5])
    p = ewald.Params(Lx=Lx, Ly=Ly, H=H, lam=3.0, alpha=6.0, rc=0.5, coulomb_k=1.0)
    e2d = ewald2d.energy_q2d(p, pos, q)
    R = 80.0
    ei = ewald2d.energy_images(p, pos, q, R) + ewald2d.disc_tail(p, pos, q, R)
    assert abs(ei - e2d) < 2e-5 * abs(e2d)


def test_ew3dc_converges_to_ewald2d_with_padding():
    rng = np.random.default_rng(3)
    Lx, Ly, H = 1.0, 1.2, 1.5
    pos = np.column_stack([rng.uniform(0, Lx, 6), rng.uniform(0, Ly, 6), rng.uniform(0.2, H - 0.2, 6)])
    q = np.array([1, -1, 1, -1, 0.5, -0.5])
    p = ewald.Params(Lx=Lx, Ly=Ly, H=H, lam=3.0, alpha=6.0, rc=0.5, coulomb_k=1.0)
    e2d = ewald2d.energy_q2d(p, pos, q)
    errs = []
    for lam in (2.0, 3.0, 6.0):
        E = ewald.energy(p.with_(lam=lam), pos, q, np.zeros((0, 3)), np.zeros(0))["total"]
        errs.append(abs(E - e2d) / abs(e2d))
    assert errs[0] > errs[1] > errs[2]
    assert errs[1] < 1e-7 and errs[2] < 1e-12
    # without the slab term the padded sum does not approach the quasi-2D energy
    E_noslab = ewald.energy(p.with_(lam=6.0, slab=False), pos, q, np.zeros((0, 3)), np.zeros(0))["total"]
    assert abs(E_noslab - e2d) > 1e-3 * abs(e2d)


def test_gaussian_electrodes_vs_image_sum():
    # EW3DC at lambda = 6 equals the quasi-2D energy to ~1e-12; the brute-force
    # image sum of point charges and Gaussians checks every kernel of Eq. (13)
    # and the Gaussian self term of Eq. (17).
    rng = np.random.default_rng(11)
    Lx, Ly, H = 1.0, 1.1, 1.2
    ion = np.column_stack([rng.uniform(0, Lx, 4), rng.uniform(0, Ly, 4), rng.uniform(0.3, H - 0.3, 4)])
    ion[0] = [0.27, 0.31, 0.08]  # close enough to an electrode for the erfc(r/eta) part to matter
    q = np.array([1.0, -1.0, 0.6, -0.2])
    ele = np.array([[0.25, 0.3, 0.0], [0.75, 0.8, 0.0], [0.2, 0.7, H], [0.7, 0.2, H]])
    Q = np.array([-0.3, -0.2, 0.1, 0.0])
    p = ewald.Params(Lx=Lx, Ly=Ly, H=H, lam=6.0, alpha=6.0, eta=0.07, rc=0.5, coulomb_k=1.0, kspace_tol=1e-18)
    E = ewald.energy(p, ion, q, ele, Q)["total"]
    pos = np.vstack([ion, ele])
    qq = np.concatenate([q, Q])
    w = np.concatenate([np.zeros(4), np.full(4, p.eta)])
    R = 80.0
    ei = ewald2d.energy_images(p, pos, qq, R, w) + ewald2d.disc_tail(p, pos, qq, R)
    assert abs(ei - E) < 1e-5 * abs(E)


# ---------------------------------------------------------------- derivatives


def test_forces_are_minus_gradient_full_ewald():
    p, ion, q, ele, side = tiny_system()
    modes = ewald.enumerate_modes(p)
    Q = np.random.default_rng(1).normal(size=len(ele)) * 0.1
    Fi, Fe = ewald.forces(p, ion, q, ele, Q, modes)
    h = 1e-5
    for i in range(len(ion)):
        for d in range(3):
            ip, im = ion.copy(), ion.copy()
            ip[i, d] += h
            im[i, d] -= h
            fd = -(ewald.energy(p, ip, q, ele, Q, modes)["total"] - ewald.energy(p, im, q, ele, Q, modes)["total"]) / (2 * h)
            assert abs(fd - Fi[i, d]) < 1e-6 * (1 + abs(Fi[i, d]))
    # one electrode coordinate as well
    for d in range(3):
        ep, em = ele.copy(), ele.copy()
        ep[4, d] += h
        em[4, d] -= h
        fd = -(ewald.energy(p, ion, q, ep, Q, modes)["total"] - ewald.energy(p, ion, q, em, Q, modes)["total"]) / (2 * h)
        assert abs(fd - Fe[4, d]) < 1e-6 * (1 + abs(Fe[4, d]))


def test_A_and_b_are_derivatives_of_energy():
    # Pins the readings of Eqs. (18)-(19): A = d2U/dQ2 (slab entry 4 pi/V) and
    # b = -dU/dQ at Q = 0 (slab entry with a minus sign), and U = 1/2 QAQ - bQ + c.
    p, ion, q, ele, side = tiny_system()
    modes = ewald.enumerate_modes(p)
    A = ewald.electrode_matrix(p, ele, modes)
    b = ewald.electrode_vector(p, ion, q, ele, modes)
    c = ewald.constant_term(p, ion, q, modes)
    rng = np.random.default_rng(4)
    Q = rng.normal(size=len(ele)) * 0.1
    U = lambda Qv: ewald.energy(p, ion, q, ele, Qv, modes)["total"]
    assert U(Q) == pytest.approx(0.5 * Q @ A @ Q - b @ Q + c, rel=1e-12, abs=1e-12)
    h = 1e-3
    n = len(ele)
    for j in range(n):
        e = np.zeros(n)
        e[j] = h
        g = (U(e) - U(-e)) / (2 * h)
        assert abs(g + b[j]) < 1e-9
    for (i, j) in [(0, 0), (0, 1), (0, 10), (4, 13), (17, 17)]:
        ei = np.zeros(n)
        ej = np.zeros(n)
        ei[i] = h
        ej[j] = h
        hess = (U(ei + ej) - U(ei - ej) - U(-ei + ej) + U(-ei - ej)) / (4 * h * h)
        assert abs(hess - A[i, j]) < 1e-7 * (1 + abs(A[i, j]))
    assert np.allclose(A, A.T, atol=1e-14 * np.max(np.abs(A)))
    assert np.min(np.linalg.eigvalsh(A)) > 0


def test_srbe_forces_are_minus_gradient_of_srbe_energy():
    p, ion, q, ele, side = tiny_system()
    modes = ewald.enumerate_modes(p)
    A = ewald.electrode_matrix(p, ele, modes)
    ks, _ = sampler.draw_kset(p, seed=9, stream=0, step=1)
    Q = np.random.default_rng(8).normal(size=len(ele)) * 0.1
    F = srbe.srbe_ion_forces(p, ks, ion, q, ele, Q)
    h = 1e-5
    for i in range(len(ion)):
        for d in range(3):
            ip, im = ion.copy(), ion.copy()
            ip[i, d] += h
            im[i, d] -= h
            fd = -(srbe.srbe_energy(p, A, ks, ip, q, ele, Q) - srbe.srbe_energy(p, A, ks, im, q, ele, Q)) / (2 * h)
            assert abs(fd - F[i, d]) < 1e-6 * (1 + abs(F[i, d]))


# ---------------------------------------------------------------- constant-potential solve


@pytest.fixture(scope="module")
def cp_system():
    p, ion, q, ele, side = tiny_system()
    modes = ewald.enumerate_modes(p)
    A = ewald.electrode_matrix(p, ele, modes)
    b = ewald.electrode_vector(p, ion, q, ele, modes)
    return p, ion, q, ele, side, A, b, cp.Solver(A)


def test_cp_neutral_and_equipotential(cp_system):
    p, ion, q, ele, side, A, b, sol = cp_system
    dpsi = 2.0
    Q, psibar = sol.solve(side, dpsi, b)
    assert abs(np.sum(Q)) < 1e-14 * np.sum(np.abs(Q))
    Psi = A @ Q - b
    neg, pos = side < 0, side > 0
    assert np.ptp(Psi[neg]) < 1e-12 and np.ptp(Psi[pos]) < 1e-12
    assert Psi[neg].mean() == pytest.approx(psibar - dpsi / 2, abs=1e-12)
    assert Psi[pos].mean() == pytest.approx(psibar + dpsi / 2, abs=1e-12)
    assert np.sum(Q[neg]) == pytest.approx(-np.sum(Q[pos]), abs=1e-14)


def test_cp_linear_in_voltage_and_gauge_invariant(cp_system):
    p, ion, q, ele, side, A, b, sol = cp_system
    Q0, _ = sol.solve(side, 0.0, b)
    Q1, _ = sol.solve(side, 1.0, b)
    Q3, _ = sol.solve(side, 3.0, b)
    assert np.allclose(Q3 - Q0, 3.0 * (Q1 - Q0), atol=1e-13)
    Qg, _ = sol.solve(side, 1.0, b + 0.37)  # any constant added to b (e.g. the Eq. (19) +dpsi)
    assert np.allclose(Qg, Q1, atol=1e-13)
    S = sol.inverse_projected()
    assert np.allclose(S @ (1.0 * cp.side_vector(side) + b), Q1, atol=1e-12)


def test_empty_capacitor():
    # No ions: the negative electrode charges negatively for dpsi > 0, the charge is
    # close to the parallel-plate value, and under neutrality it does not depend on
    # the vacuum padding (Sec. 2, after Eq. (11)).
    p, ion, q, ele, side = tiny_system()
    outs = []
    for lam in (3.0, 6.0):
        pl = p.with_(lam=lam)
        A = ewald.electrode_matrix(pl, ele)
        Q, _ = cp.Solver(A).solve(side, 2.0, np.zeros(len(ele)))
        outs.append(Q)
    qneg = np.sum(outs[0][side < 0])
    assert qneg < 0
    plate = p.Lx * p.Ly * 2.0 / (4 * np.pi * p.coulomb_k * p.H)
    assert abs(-qneg - plate) < 0.15 * plate
    assert np.max(np.abs(outs[0] - outs[1])) < 1e-6 * np.max(np.abs(outs[0]))


# ---------------------------------------------------------------- SRBE structure and statistics


def test_srbe_deterministic_part_is_exact():
    # With an empty batch only the modes of I remain; they must equal the full
    # sum restricted to I, independently of any seed.
    p, ion, q, ele, side = tiny_system(M=6)
    mI = srbe.deterministic_modes(p.M)
    bI = srbe.srbe_b_fourier(p, np.zeros((0, 3)), ion, q, ele)
    S1 = ewald.structure_factor(p, mI, ion, q)
    k2 = np.sum(ewald.kvectors(p, mI) ** 2, axis=1)
    ref = np.zeros(len(ele))
    for t in range(len(mI)):
        ref -= ewald.ewald_weight(p, k2[t]) * np.real(np.exp(-1j * ele @ ewald.kvectors(p, mI[t:t + 1])[0]) * S1[t])
    assert np.allclose(bI, p.coulomb_k * ref, rtol=0, atol=1e-13)


@pytest.mark.parametrize("rc", [0.6, 0.8])  # 0.6: minimum image; 0.8 > L/2: several images per pair
def test_sampled_targets_match_the_full_functions(rc):
    # The sampled-target forms (for systems too large to evaluate every target) give
    # the full functions' values at the sampled targets, and the particle-chunked
    # structure factor the one-chunk sum: the same terms, summed in another order.
    import dataclasses
    p, ion, q, ele, side = tiny_system(n_ion=12)
    p = dataclasses.replace(p, rc=rc)
    ks, _ = sampler.draw_kset(p, seed=3, stream=0, step=1)
    Q = np.random.default_rng(2).normal(size=len(ele)) * 0.05
    ii = np.array([7, 0, 11, 3])
    ie = np.array([17, 2, 9])
    F = srbe.srbe_ion_forces(p, ks, ion, q, ele, Q)
    b = srbe.srbe_b(p, ks, ion, q, ele)
    assert np.allclose(srbe.srbe_ion_forces_at(p, ks, ion, q, ele, Q, ii), F[ii], rtol=1e-13, atol=1e-13)
    assert np.allclose(srbe.srbe_b_at(p, ks, ion, q, ele, ie), b[ie], rtol=1e-13, atol=1e-13)
    m, _ = srbe._combined(p, ks)
    assert np.allclose(ewald.structure_factor(p, m, ion, q, pchunk=5), ewald.structure_factor(p, m, ion, q),
                       rtol=0, atol=1e-13)


def test_momentum_conserved_per_sample(cp_system):
    p, ion, q, ele, side, A, b, sol = cp_system
    ks, _ = sampler.draw_kset(p, seed=5, stream=0, step=2)
    bs = srbe.srbe_b(p, ks, ion, q, ele)
    Q, _ = sol.solve(side, 2.0, bs)
    Fi = srbe.srbe_ion_forces(p, ks, ion, q, ele, Q)
    Fe = srbe.srbe_ele_forces(p, ks, ion, q, ele, Q)
    tot = Fi.sum(axis=0) + Fe.sum(axis=0)
    assert np.max(np.abs(tot)) < 1e-12 * np.max(np.abs(Fi))


def test_srbe_unbiased():
    # Theorems 3.1, 3.2: b*_F and F*_F (fixed Q) have the full Ewald sums as mean.
    p, ion, q, ele, side = tiny_system(M=3, P=10, tol=1e-16)
    modes = ewald.enumerate_modes(p)
    Q = np.random.default_rng(2).normal(size=len(ele)) * 0.1
    k2 = np.sum(ewald.kvectors(p, modes) ** 2, axis=1)
    w = ewald.ewald_weight(p, k2)
    S1 = ewald.structure_factor(p, modes, ion, q)
    b_ref = -p.coulomb_k * ewald.fourier_potential(p, modes, w * S1, ele)
    S = S1 + ewald.structure_factor(p, modes, ele, Q)
    F_ref = -p.coulomb_k * q[:, None] * ewald.fourier_gradient_term(p, modes, w * S, ion)
    B = 3000
    bs = np.zeros((B, len(ele)))
    Fs = np.zeros((B, len(ion), 3))
    for t in range(B):
        ks, _ = sampler.draw_kset(p, seed=77, stream=0, step=t)
        bs[t] = srbe.srbe_b_fourier(p, ks, ion, q, ele)
        Fs[t] = srbe.srbe_force_fourier(p, ks, ion, q, ele, Q)
    zb = (bs.mean(0) - b_ref) / (bs.std(0) / np.sqrt(B))
    zF = (Fs.mean(0) - F_ref) / (Fs.std(0) / np.sqrt(B))
    assert np.max(np.abs(zb)) < 5.0
    assert np.max(np.abs(zF)) < 5.0
    # variance shrinks like 1/P
    bs4 = np.array([srbe.srbe_b_fourier(p.with_(P=40), sampler.draw_kset(p.with_(P=40), 78, 0, t)[0], ion, q, ele)
                    for t in range(600)])
    ratio = bs[:600].var(0).mean() / bs4.var(0).mean()
    assert 2.5 < ratio < 6.0


def test_srbe_variance_drops_with_deterministic_modes():
    # Sec. 3's variance bound for the electrode-potential fluctuation depends on the
    # smallest sampled mode, omega = min(2 pi / max(Lx, Ly), 2 pi (M + 1) / Lz): taking
    # the kz modes up to M out of the sample (the symmetry-preserving part) shrinks
    # the variance of b* at fixed P, most for M > 0 against M = 0 (the remark after
    # the bound).  Measured here 1 : 0.31 : 0.16 for M = 0, 1, 3.
    p, ion, q, ele, side = tiny_system(M=3, P=10, tol=1e-16)
    var = {}
    for M in (0, 1, 3):
        pm = p.with_(M=M)
        bs = np.array([srbe.srbe_b_fourier(pm, sampler.draw_kset(pm, 91, 0, t)[0], ion, q, ele) for t in range(600)])
        var[M] = bs.var(0).mean()
    assert var[1] < 0.6 * var[0]
    assert var[3] < 0.7 * var[1]


def test_srbe_weight_normalisation():
    # E[sum_l w_l] over batches must equal sum over L_k \ I of 4 pi exp(-k^2/4a^2)/(V k^2):
    # pins the G/P factor and the 4 pi/(V k^2) weight of Eq. (24) with no cancellation.
    p = ewald.Params(Lx=1.2, Ly=1.3, H=1.5, lam=3.0, alpha=4.0, M=3, P=16)
    modes = ewald.enumerate_modes(p, tol=1e-30)
    modes = modes[sampler.valid(p, modes)]
    exact = np.sum(ewald.ewald_weight(p, np.sum(ewald.kvectors(p, modes) ** 2, axis=1)))
    B = 4000
    tot = np.array([srbe.mode_weights(p, sampler.draw_kset(p, 3, 0, t)[0])[3].sum() for t in range(B)])
    z = (tot.mean() - exact) / (tot.std() / np.sqrt(B))
    assert abs(z) < 5.0
    assert abs(tot.mean() / exact - 1.0) < 0.02


def small_cell(seed=4):
    """0.8 x 0.8 x 1.0 cell, two 2 x 2 Gaussian walls and four ions: few enough modes to
    evaluate the estimator once per mode of the whole reciprocal lattice."""
    rng = np.random.default_rng(seed)
    Lx, Ly, H = 0.8, 0.8, 1.0
    g = (np.arange(2) + 0.5) * 0.4
    X, Y = np.meshgrid(g, g, indexing="ij")
    wall = np.column_stack([X.ravel(), Y.ravel()])
    ele = np.vstack([np.column_stack([wall, np.zeros(4)]), np.column_stack([wall, np.full(4, H)])])
    ion = np.column_stack([rng.uniform(0, Lx, 4), rng.uniform(0, Ly, 4), rng.uniform(0.3, H - 0.3, 4)])
    q = np.array([0.8, -0.8, 0.5, -0.5])
    p = ewald.Params(Lx=Lx, Ly=Ly, H=H, lam=3.0, alpha=5.0, eta=0.08, rc=0.4, coulomb_k=1.44, M=3, P=1,
                     kspace_tol=1e-10)
    Q = rng.normal(size=len(ele)) * 0.1
    return p, ion, q, ele, Q


def test_srbe_energy_expectation_over_every_mode_is_the_full_ewald_energy():
    # E* at fixed Q (reading R6) is the deterministic part plus (1/P) sum_l of a term of the
    # sampled mode, so its expectation under the sampling law exp(-k^2/4a^2)/G on L_k \ I
    # (Eqs. (26)-(27), Theorems 3.1-3.2) can be taken exactly: weight the one-mode estimate
    # E*({k}) of every mode by its probability, and give the probability mass beyond the
    # truncated lattice to the empty-batch estimate (the deterministic part alone).  That
    # must be the complete energy U_c = 1/2 Q^T A Q - b^T Q + c of Eqs. (13), (16), (17),
    # with every position-independent term (the ion self term -a/sqrt(pi) sum q^2, the
    # Gaussian self term, the slab term) included: a finite-difference force check
    # cancels those terms, this identity does not.
    p, ion, q, ele, Q = small_cell()
    modes = ewald.enumerate_modes(p)
    A = ewald.electrode_matrix(p, ele, modes)
    mv = modes[sampler.valid(p, modes)]
    prob = np.exp(-np.sum(ewald.kvectors(p, mv) ** 2, axis=1) / (4 * p.alpha ** 2)) / srbe.normaliser_G(p)
    assert 1.0 - 1e-8 < prob.sum() < 1.0
    expect = sum(pr * srbe.srbe_energy(p, A, k[None, :], ion, q, ele, Q) for k, pr in zip(mv, prob))
    expect += (1.0 - prob.sum()) * srbe.srbe_energy(p, A, np.zeros((0, 3)), ion, q, ele, Q)
    full = ewald.energy(p, ion, q, ele, Q, modes)["total"]
    assert abs(expect - full) < 1e-13 * abs(full)
    # the same identity for c* alone (no electrode charges): c of Eq. (5)
    expect_c = sum(pr * srbe.srbe_constant(p, k[None, :], ion, q) for k, pr in zip(mv, prob))
    expect_c += (1.0 - prob.sum()) * srbe.srbe_constant(p, np.zeros((0, 3)), ion, q)
    c = ewald.constant_term(p, ion, q, modes)
    assert abs(expect_c - c) < 1e-13 * abs(c)


def test_srbe_energy_parts():
    # The split of E* into real, Fourier, self and slab parts, computed from each part's own
    # definition: (1) the parts add up to E* = 1/2 Q^T A Q - b*^T Q + c* for any sample;
    # (2) the SRBE leaves the real, self and slab parts of U_c (Eqs. (13), (17)) untouched,
    # so they equal the complete energy's own parts exactly, and (3) the Fourier part's
    # expectation over every mode (as in the pin above) is the complete Fourier energy
    # of Eq. (16).
    p, ion, q, ele, Q = small_cell()
    modes = ewald.enumerate_modes(p)
    A = ewald.electrode_matrix(p, ele, modes)
    full = ewald.energy(p, ion, q, ele, Q, modes)
    mv = modes[sampler.valid(p, modes)]
    prob = np.exp(-np.sum(ewald.kvectors(p, mv) ** 2, axis=1) / (4 * p.alpha ** 2)) / srbe.normaliser_G(p)
    expect = 0.0
    for k, pr in zip(mv, prob):
        parts = srbe.srbe_energy_parts(p, k[None, :], ion, q, ele, Q, modes)
        expect += pr * parts["fourier"]
    empty = srbe.srbe_energy_parts(p, np.zeros((0, 3)), ion, q, ele, Q, modes)
    expect += (1.0 - prob.sum()) * empty["fourier"]
    assert abs(expect - full["fourier"]) < 1e-13 * abs(full["total"])
    kset = np.array([mv[3], mv[7], mv[3]])
    parts = srbe.srbe_energy_parts(p, kset, ion, q, ele, Q, modes)
    E = srbe.srbe_energy(p, A, kset, ion, q, ele, Q)
    assert abs(parts["total"] - E) < 1e-13 * abs(E)
    for name in ("real", "self", "slab"):
        assert abs(parts[name] - full[name]) < 1e-13 * abs(full["total"]), name
        assert abs(full[name]) > 1e-4 * abs(full["total"]), name  # each part is really there


def test_srbe_energy_sample_mean_is_the_full_ewald_energy():
    # The same statement through the sampler itself: the mean of E* over 2000 batches drawn
    # by the Metropolis chain (fixed Q) equals the complete energy within 5 standard errors.
    p, ion, q, ele, side = tiny_system(M=3, P=10, tol=1e-16)
    modes = ewald.enumerate_modes(p)
    A = ewald.electrode_matrix(p, ele, modes)
    Q = np.random.default_rng(6).normal(size=len(ele)) * 0.1
    full = ewald.energy(p, ion, q, ele, Q, modes)["total"]
    B = 2000
    Es = np.array([srbe.srbe_energy(p, A, sampler.draw_kset(p, 41, 0, t)[0], ion, q, ele, Q) for t in range(B)])
    z = (Es.mean() - full) / (Es.std() / np.sqrt(B))
    assert abs(z) < 5.0


# ---------------------------------------------------------------- virial (pressure) tensor


def _strain_energy_pins_system():
    rng = np.random.default_rng(21)
    p, ion, q, ele, Q = small_cell(seed=9)
    return p, ion, q, ele, Q, rng


def test_fourier_virial_is_minus_the_strain_derivative():
    # Under r -> (I + e) r with the box strained alike, fractional coordinates and S(k)
    # stay, k -> (I + e)^-T k and V -> det(I + e) V: U_F(e) = 1/2 sum w(k(e), V(e)) |S|^2.
    # Its central finite difference in each of the nine strain components must be
    # minus the analytic virial (which is symmetric).
    from oracle import virial
    p, ion, q, ele, Q, _ = _strain_energy_pins_system()
    modes = ewald.enumerate_modes(p)
    S = ewald.structure_factor(p, modes, ion, q) + ewald.structure_factor(p, modes, ele, Q)
    k0 = ewald.kvectors(p, modes)

    def UF(eps):
        F = np.eye(3) + eps
        k = k0 @ np.linalg.inv(F)  # rows: (F^-T k)^T = k^T F^-1
        k2 = np.sum(k * k, axis=1)
        V = p.V * np.linalg.det(F)
        return 0.5 * np.sum(4 * np.pi * np.exp(-k2 / (4 * p.alpha ** 2)) / (V * k2) * np.abs(S) ** 2)

    k2 = np.sum(k0 ** 2, axis=1)
    W = virial.fourier_virial(p, modes, ewald.ewald_weight(p, k2), S)
    h = 1e-6
    for a in range(3):
        for b in range(3):
            e = np.zeros((3, 3))
            e[a, b] = h
            fd = -(UF(e) - UF(-e)) / (2 * h)
            assert abs(fd - W[a, b]) < 1e-7 * np.max(np.abs(W)), (a, b, fd, W[a, b])
    assert np.max(np.abs(W - W.T)) < 1e-12 * np.max(np.abs(W))


def test_real_and_slab_virial_are_minus_the_strain_derivative():
    # Every pair vector within rc stretches with the strain, the kernels do not; the
    # slab term changes through V and M_z.  Finite differences of the strained sums.
    from oracle import virial
    p, ion, q, ele, Q, _ = _strain_energy_pins_system()
    pos = np.concatenate([ion, ele])
    qq = np.concatenate([q, Q])
    kind = np.array(["i"] * len(ion) + ["g"] * len(ele))
    pairs = []
    for i in range(len(pos)):
        for j in range(i + 1, len(pos)):
            d = pos[i] - pos[j]
            d[0] -= p.Lx * np.round(d[0] / p.Lx)
            d[1] -= p.Ly * np.round(d[1] / p.Ly)
            if np.linalg.norm(d) < p.rc:
                K = {"ii": ewald.kernel_ion_ion, "ig": ewald.kernel_ion_gauss, "gi": ewald.kernel_ion_gauss,
                     "gg": ewald.kernel_gauss_gauss}[kind[i] + kind[j]]
                pairs.append((d, qq[i] * qq[j], K))
    assert len(pairs) > 10

    def UN(eps):
        return sum(c * K(p, np.linalg.norm((np.eye(3) + eps) @ d)) for d, c, K in pairs)

    W = virial.real_virial(p, ion, q, ele, Q)
    Mz = q @ ion[:, 2] + Q @ ele[:, 2]

    def Us(eps):
        F = np.eye(3) + eps
        return 2 * np.pi / (p.V * np.linalg.det(F)) * (F[2, 2] * Mz) ** 2

    Ws = virial.slab_virial(p, ion, q, ele, Q)
    h = 1e-6
    for a in range(3):
        for b in range(3):
            e = np.zeros((3, 3))
            e[a, b] = h
            fd = -(UN(e) - UN(-e)) / (2 * h)
            assert abs(fd - W[a, b]) < 1e-7 * np.max(np.abs(W)), (a, b, fd, W[a, b])
        e = np.zeros((3, 3))
        e[a, a] = h
        fd = -(Us(e) - Us(-e)) / (2 * h)
        assert abs(fd - Ws[a, a]) < 1e-7 * abs(Ws[0, 0])


def test_virial_trace_is_the_coulomb_energy():
    # Point charges alone: the complete Coulomb energy is homogeneous of degree -1 in
    # the lengths, so the trace of its virial equals the energy (independently of how
    # Ewald splits it).  alpha rc = 6 keeps the real-space cut below 1e-16.
    from oracle import virial
    rng = np.random.default_rng(8)
    p = ewald.Params(Lx=2.4, Ly=2.4, H=2.0, lam=3.0, alpha=5.0, eta=0.05, rc=1.2, coulomb_k=1.44,
                     kspace_tol=1e-16)
    n = 16
    ion = np.column_stack([rng.uniform(0, p.Lx, n), rng.uniform(0, p.Ly, n), rng.uniform(0.3, p.H - 0.3, n)])
    q = np.where(np.arange(n) % 2 == 0, 0.8, -0.8)
    none = np.zeros((0, 3))
    W = virial.complete_virial(p, ion, q, none, np.zeros(0))
    U = ewald.energy(p, ion, q, none, np.zeros(0))["total"]
    assert abs(W[0] + W[1] + W[2] - U) < 1e-10 * abs(U), (W[:3].sum(), U)


def test_srbe_virial_expectation_over_every_mode_is_the_complete_virial():
    # As for E*: weighting the one-mode estimate by each mode's sampling probability
    # (the empty-batch estimate for the mass beyond the truncation) gives the virial of
    # the complete energy, every component, to 1e-13.
    from oracle import virial
    p, ion, q, ele, Q = small_cell()
    modes = ewald.enumerate_modes(p)
    full = virial.complete_virial(p, ion, q, ele, Q, modes)
    mv = modes[sampler.valid(p, modes)]
    prob = np.exp(-np.sum(ewald.kvectors(p, mv) ** 2, axis=1) / (4 * p.alpha ** 2)) / srbe.normaliser_G(p)
    expect = sum(pr * virial.srbe_virial(p, k[None, :], ion, q, ele, Q) for k, pr in zip(mv, prob))
    expect = expect + (1.0 - prob.sum()) * virial.srbe_virial(p, np.zeros((0, 3)), ion, q, ele, Q)
    assert np.max(np.abs(expect - full)) < 1e-13 * np.max(np.abs(full))
    assert np.max(np.abs(full[3:])) > 1e-3 * np.max(np.abs(full))  # shear components present


# ---------------------------------------------------------------- Langevin update (Sec. 3)


def test_langevin_noiseless_step_is_explicit_euler():
    # beta -> infinity removes the noise: the update is r + v dt, v + (F - gamma v) dt / m
    rng = np.random.default_rng(3)
    n = 50
    pos = np.column_stack([rng.uniform(0, 2, n), rng.uniform(0, 3, n), rng.uniform(1, 4, n)])
    vel, F, m = rng.normal(size=(n, 3)) * 0.01, rng.normal(size=(n, 3)), rng.uniform(1, 3, n)
    dt, gamma = 1e-3, 2.0
    r, v = langevin.euler_maruyama(pos, vel, F, m, gamma, np.inf, dt, 2.0, 3.0, 0.5, 4.5, 7, 0)
    assert np.allclose(r, pos + vel * dt, rtol=0, atol=1e-15)
    assert np.allclose(v, vel + (F - gamma * vel) * dt / m[:, None], rtol=0, atol=1e-15)


def test_langevin_noise_has_the_fluctuation_dissipation_variance():
    # at zero force and velocity the velocity change is sqrt(2 gamma / beta) dW / m, dW ~ N(0, dt):
    # variance 2 gamma dt / (beta m^2) per component, uncorrelated across components
    n = 200000
    m, gamma, beta, dt = 2.0, 3.0, 0.5, 1e-2
    pos = np.tile([1.0, 1.0, 2.0], (n, 1))
    _, v = langevin.euler_maruyama(pos, np.zeros((n, 3)), np.zeros((n, 3)), np.full(n, m), gamma, beta, dt,
                                   4.0, 4.0, 0.0, 4.0, 11, 5)
    var = 2.0 * gamma * dt / (beta * m * m)
    assert np.allclose(v.var(axis=0) / var, 1.0, atol=0.02)
    assert np.allclose(v.mean(axis=0) / np.sqrt(var), 0.0, atol=0.02)
    c = np.corrcoef(v.T)
    assert np.all(np.abs(c[np.triu_indices(3, 1)]) < 0.02)


def test_langevin_walls_reflect_and_wrap():
    # ion 0 leaves through x = 0 and z = zlo, ion 1 through x = Lx, y = Ly and z = zhi
    pos = np.array([[0.005, 0.2, 0.52], [1.995, 2.995, 4.45]])
    vel = np.array([[-1.0, -1.0, -10.0], [1.0, 1.0, 10.0]])
    r, v = langevin.euler_maruyama(pos, vel, np.zeros((2, 3)), np.ones(2), 0.0, np.inf, 0.01, 2.0, 3.0, 0.5, 4.5,
                                   1, 0)
    assert np.allclose(r[:, 0], [2.0 - 0.005, 0.005], atol=1e-14)
    assert np.allclose(r[:, 1], [0.19, 0.005], atol=1e-14)
    assert np.allclose(r[:, 2], [2 * 0.5 - 0.42, 2 * 4.5 - 4.55], atol=1e-14)
    assert np.allclose(v[:, 2], [10.0, -10.0]) and np.allclose(v[:, :2], vel[:, :2])


def test_langevin_large_overshoot_lands_inside():
    # a step that crosses the electrolyte more than once is folded back by repeated
    # reflections: the mirror images of the straight path in the walls, v_z flipped once
    # per reflection
    zlo, zhi = 0.5, 4.5
    W = zhi - zlo
    z0 = np.array([4.0, 1.0, 2.0, 3.0, 1.0])
    vz = np.array([9.0, -30.0, 10.0 * W, -1e4, 0.0])  # dt = 0.1: 0.4 past zhi by 0.5 W, ...
    pos = np.column_stack([np.ones(5), np.ones(5), z0])
    vel = np.column_stack([np.zeros(5), np.zeros(5), vz])
    r, v = langevin.euler_maruyama(pos, vel, np.zeros((5, 3)), np.ones(5), 0.0, np.inf, 0.1, 2.0, 2.0, zlo, zhi, 1, 0)
    assert np.all((r[:, 2] >= zlo) & (r[:, 2] <= zhi))
    # brute force: reflect one wall at a time until inside
    for z, u, zr, vr in zip(z0 + 0.1 * vz, vz, r[:, 2], v[:, 2]):
        n = 0
        while z < zlo or z > zhi:
            z = 2 * zlo - z if z < zlo else 2 * zhi - z
            n += 1
        assert zr == pytest.approx(z, abs=1e-9)
        assert vr == (-u if n % 2 else u)


# ---------------------------------------------------------------- short-range force field (dynamics)


def _ff():
    return dict(wca_eps=0.05, wca_sigma=0.3, wall_eps=0.2, wall_sigma=0.35, wall_zlo=0.5, wall_zhi=3.5, bond_k=500.0)


def test_forcefield_terms_closed_forms():
    from oracle import forcefield
    ff = _ff()
    s = ff["wca_sigma"]
    u, _ = forcefield.wca(0.05, s, s)
    assert u == pytest.approx(0.05, rel=1e-14)  # 4 eps (1 - 1) + eps
    rc = 2 ** (1 / 6) * s
    u, du = forcefield.wca(0.05, s, rc * (1 - 1e-12))
    assert abs(u) < 1e-12 and abs(du) < 1e-9  # continuous with zero force at the cut
    dmin = (2 / 5) ** (1 / 6) * ff["wall_sigma"]
    u, du = forcefield.wall93(0.2, ff["wall_sigma"], dmin * (1 - 1e-12))
    assert abs(u) < 1e-12 and abs(du) < 1e-9  # cut and shifted at the minimum
    u, du = forcefield.wall93(0.2, ff["wall_sigma"], 0.5 * dmin)
    assert u > 0 and du < 0  # repulsive


def test_forcefield_forces_are_minus_gradient():
    from oracle import forcefield
    # sites on a jittered 0.31 nm grid (some pairs inside the WCA range, none closer than
    # ~0.26 nm), within the walls' reach at both ends, x and y across the periodic boundary
    rng = np.random.default_rng(11)
    Lx = Ly = 1.24
    g = np.array([[ix, iy, iz] for ix in range(2) for iy in range(2) for iz in range(4)], dtype=float)[:14]
    pos = g * 0.31 + rng.uniform(-0.02, 0.02, (14, 3)) + np.array([1.1, 0.05, 0.0])
    pos[:, 2] = np.where(g[:, 2] < 2, 0.75 + 0.31 * g[:, 2], 3.25 - 0.31 * (g[:, 2] - 2)) + rng.uniform(-0.02, 0.02, 14)
    pos[:, :2] %= Lx
    n = len(pos)
    mol = np.array([0, 0, 0, 1, 2, 3, 4, 4, 5, 6, 7, 8, 9, 10])
    bonds = [(0, 1, 0.3), (1, 2, 0.3), (0, 2, 0.52), (6, 7, 0.25)]
    ff = _ff()
    F = forcefield.forces(pos, mol, bonds, ff, Lx, Ly)
    assert np.any(F != 0)
    h = 1e-6
    for i in range(n):
        for d in range(3):
            p1, p0 = pos.copy(), pos.copy()
            p1[i, d] += h
            p0[i, d] -= h
            fd = -(forcefield.energy(p1, mol, bonds, ff, Lx, Ly) - forcefield.energy(p0, mol, bonds, ff, Lx, Ly)) / (2 * h)
            assert abs(fd - F[i, d]) < 1e-5 * (1 + abs(F[i, d]))
    # without walls the pair and bond forces cancel (Newton's third law)
    ffw = dict(ff, wall_eps=0.0)
    assert np.max(np.abs(forcefield.forces(pos, mol, bonds, ffw, Lx, Ly).sum(axis=0))) < 1e-10


def test_langevin_update_orderings_on_a_harmonic_oscillator():
    # noiseless, frictionless one-step maps of x'' = -omega^2 x (F = -k x, m = 1): the
    # printed ordering (r + v^n dt) has determinant 1 + (omega dt)^2, so it gains energy
    # every step; the symplectic ordering (r + v^{n+1} dt) has determinant 1 exactly
    k, dt = 400.0, 0.01
    def step(x, v, sym):
        r, u = langevin.euler_maruyama(np.array([[1.0, 1.0, x]]), np.array([[0.0, 0.0, v]]),
                                       np.array([[0.0, 0.0, -k * x]]), np.ones(1), 0.0, np.inf, dt, 5.0, 5.0,
                                       -1e3, 1e3, 1, 0, symplectic=sym)
        return r[0, 2], u[0, 2]
    for sym, det in ((False, 1.0 + k * dt * dt), (True, 1.0)):
        a = step(1.0, 0.0, sym)
        b = step(0.0, 1.0, sym)
        assert a[0] * b[1] - a[1] * b[0] == pytest.approx(det, rel=1e-13)
