"""The lattice charge solve (SRBE_FLAG_LATTICE_SOLVE) against the oracle's dense solve.

With both electrode walls complete rectangular lattices, A (Eq. (18)) is
block-circulant and the charge update of Eqs. (9)-(11) runs per lattice Fourier
mode.  Each case takes full steps of a lattice handle and compares b*, Q, psibar,
the ion forces and E* with the FP64 oracle (dense A from ``ewald.electrode_matrix``,
``cp.Solver``) on the same sample, to the tolerances of test_gpu_step.py (FP64:
1e-11 relative max-norm; FP32: force relative RMS <= 1e-5, b and Q <= 3e-5).

Cases (rc is moved off the lattice distances: with sites exactly rc apart, the dense
build's rounded coordinate differences put each such pair on either side of the
cutoff, A is then not exactly block-circulant, and the two solves differ by terms of
the size of the real-space kernel at rc, ~1e-8 of Q here):

* the tiny slab with rc = 1.19 nm: two 12 x 12 square walls (0.2 nm) aligned above
  each other, three replicas of one placement at different voltages and seeds;
* a rectangular, AB-shifted pair: 10 x 8 sites of spacing 0.3 x 0.35 nm per wall in
  a 3.0 x 2.8 x 6 nm cell, the upper wall shifted by half a cell in x and y, 150
  ions by RSA, rc = 1.15 nm.

Also: a captured graph of a lattice step reproduces the eager step bit for bit, and
electrodes that are not two lattices (the honeycomb layers of the paper-shaped cell)
are refused with SRBE_EINVAL.
"""

import numpy as np
import pytest

from helpers import forces_from_soa, gpu_inputs, oracle_params, oracle_solver, oracle_step, rel_inf, rel_rms

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SEEDS = [2000, 31, 77]
DPSI = [2.0, 0.5, 3.0]
STEP = 4


def shifted_pair(seed=1500):
    from paper_2509_24742_amd import workloads as wl
    rng = np.random.default_rng(seed)
    Lx, Ly, H = 3.0, 2.8, 6.0
    nx, ny = 10, 8
    gx, gy = (np.arange(nx) + 0.5) * (Lx / nx), (np.arange(ny) + 0.5) * (Ly / ny)
    X, Y = np.meshgrid(gx, gy, indexing="ij")
    lo = np.column_stack([X.ravel(), Y.ravel(), np.zeros(nx * ny)])
    hi = np.column_stack([(X.ravel() + 0.5 * Lx / nx) % Lx, (Y.ravel() + 0.5 * Ly / ny) % Ly, np.full(nx * ny, H)])
    ele = np.vstack([lo, hi])
    side = np.array([-1] * (nx * ny) + [1] * (nx * ny), dtype=np.int8)
    ion = wl._rsa_sites(rng, 150, Lx, Ly, 0.4, H - 0.4, 0.3)
    q = np.array([0.78] * 75 + [-0.78] * 75)
    params = dict(Lx=Lx, Ly=Ly, H=H, lam=3.0, alpha=3.0, eta=1.0 / 19.79, rc=1.2, coulomb_k=wl.COULOMB_K, M=8, P=80)
    params["rc"] = 1.15
    return dict(params=params, ion_pos=ion, ion_q=q, ele_pos=ele, ele_side=side)


def build(w):
    import paper_2509_24742_amd as srbe_amd
    wp = dict(w["params"], kspace_tol=1e-16)
    p = oracle_params(wp)
    solver = oracle_solver(p, w["ele_pos"])
    sysm = srbe_amd.System(wp, w["ele_pos"], w["ele_side"], flags=srbe_amd.SRBE_FLAG_LATTICE_SOLVE)
    refs = [oracle_step(p, solver, s, STEP, w["ion_pos"], w["ion_q"], w["ele_pos"], w["ele_side"], d)
            for s, d in zip(SEEDS, DPSI)]
    inputs = gpu_inputs([w["ion_pos"]] * 3, [w["ion_q"]] * 3, DPSI, SEEDS)
    return dict(sys=sysm, refs=refs, inputs=inputs, n=len(w["ele_side"]))


@pytest.fixture(scope="module", params=["tiny", "shifted"])
def case(request):
    from paper_2509_24742_amd import workloads as wl
    if request.param == "tiny":
        w = wl.tiny_slab()
        w["params"] = dict(w["params"], rc=1.19)
    else:
        w = shifted_pair()
    c = build(w)
    c["name"] = request.param
    yield c
    c["sys"].close()


def check(c, precision, off, out):
    n = c["n"]
    for r, ref in enumerate(c["refs"]):
        F = forces_from_soa(out["F"], off, r)
        b = out["b"].cpu().numpy()[r * n:(r + 1) * n]
        Q = out["Q"].cpu().numpy()[r * n:(r + 1) * n]
        psibar, E = float(out["psibar"][r]), float(out["E"][r])
        print(f"{c['name']} precision {precision} replica {r}: Q {rel_inf(Q, ref['Q']):.2e} max, "
              f"F {rel_rms(F, ref['F']):.2e} rms, E {abs(E - ref['E']) / abs(ref['E']):.2e}", flush=True)
        if precision == 0:
            assert rel_inf(Q, ref["Q"]) < 1e-11, r
            assert abs(psibar - ref["psibar"]) < 1e-11 * abs(ref["psibar"]), r
            assert rel_inf(b, ref["b"]) < 1e-11 and rel_inf(F, ref["F"]) < 1e-11, r
            assert abs(E - ref["E"]) < 1e-11 * abs(ref["E"]), r
        else:
            assert rel_rms(F, ref["F"]) < 1e-5, r
            assert rel_rms(b, ref["b"]) < 3e-5 and rel_rms(Q, ref["Q"]) < 3e-5, r
        assert abs(np.sum(Q)) < 1e-12 * np.sum(np.abs(Q)), r


@pytest.mark.parametrize("precision", [0, 1])
def test_lattice_solve_matches_dense_oracle(case, precision):
    from paper_2509_24742_amd import binding
    off, xyz, q, dp, sd = case["inputs"]
    out = case["sys"].step(off, xyz, q, dp, sd, STEP, precision=precision)
    torch.cuda.synchronize()
    assert binding.srbe_sync_status(case["sys"].h) == 0, binding.srbe_last_error(case["sys"].h)
    check(case, precision, off, out)


def test_lattice_graph_replay_is_bitwise_eager(case):
    from paper_2509_24742_amd import binding
    off, xyz, q, dp, sd = case["inputs"]
    sysm = case["sys"]
    eager = sysm.step(off, xyz, q, dp, sd, STEP, precision=1)
    gr = sysm.capture(off, xyz, q, dp, sd, STEP, precision=1)
    try:
        gr.launch()
        torch.cuda.synchronize()
        assert binding.srbe_sync_status(sysm.h) == 0, binding.srbe_last_error(sysm.h)
        for key in ("Q", "psibar", "F", "b", "E"):
            assert torch.equal(gr.out[key], eager[key]), key
    finally:
        gr.close()


def test_not_a_lattice_is_refused():
    import paper_2509_24742_amd as srbe_amd
    from paper_2509_24742_amd import binding, workloads as wl
    w = wl.paper_cell()
    with pytest.raises(binding.SrbeError) as ei:
        srbe_amd.System(w["params"], w["ele_pos"], w["ele_side"], flags=srbe_amd.SRBE_FLAG_LATTICE_SOLVE)
    assert ei.value.code == binding.SRBE_EINVAL
