"""Large replicas and fine cell grids: the multi-block cell sort.

Replicas of more than 8192 ions, and boxes whose real-space grid has more than 2048
cells, are cell-sorted by the multi-block counting sort (so are the electrodes at
set-up beyond those sizes).  Its order is the one-block sort's, so every later pass
runs unchanged.  Each case compares b* and the ion forces at fixed electrode charges
with the FP64 oracle on the device-drawn k-set, to the tolerances of test_gpu_step.py
(FP64: 1e-11 relative max-norm; FP32: force relative RMS <= 1e-5, b <= 3e-5).  The
handles are built without the CP solve: the electrode matrix of these boxes is beyond
what the oracle builds in seconds.  A graph replay of the same step must reproduce
the eager step bit for bit.

Cases (square-wall slabs of the large-system recipe, ions at 10 per nm^3 or below):

* tall: one replica of 10,000 ions in 4.8 x 4.8 x 48 nm (1,920 cells): the ions take
  the multi-block sort for their count; the 1,152 electrodes take the one-block sort.
* wide: two replicas of 3,000 and 1,502 ions (ragged tiles) in 13.6 x 13.6 x 12 nm
  with 2 x 68 x 68 = 9,248 electrodes (3,630 cells): ions and electrodes both take
  the multi-block sort, for the grid (and the electrodes also for their count).
* full size: the large slab of 917,504 ions and 131,072 electrodes (155,625 cells),
  checked at 64 sampled ions and electrodes against stored oracle values.
"""

import numpy as np
import pytest

from helpers import forces_from_soa, gpu_inputs, oracle_params, rel_inf, rel_rms
from oracle import sampler, srbe

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

STEP = 3

CASES = {
    "tall": dict(n_side=24, Lx=4.8, H=48.0, reps=[(10000, 1500)], dpsi=[2.0], seeds=[71]),
    "wide": dict(n_side=68, Lx=13.6, H=12.0, reps=[(3000, 1501), (1502, 1502)], dpsi=[1.0, 3.5], seeds=[72, 73]),
}


def build_case(name):
    import paper_2509_24742_amd as srbe_amd
    from paper_2509_24742_amd import workloads as wl
    c = CASES[name]
    ws = [wl.large_slab(n_side=c["n_side"], n_ion=n, Lx=c["Lx"], H=c["H"], M=20, P=100, seed=s) for n, s in c["reps"]]
    wp = dict(ws[0]["params"], kspace_tol=1e-16)
    p = oracle_params(wp)
    ele, side = ws[0]["ele_pos"], ws[0]["ele_side"]
    rng = np.random.default_rng(9)
    Qs = [side * 0.004 + 0.001 * rng.normal(size=len(side)) for _ in ws]
    sysm = srbe_amd.System(wp, ele, side, flags=srbe_amd.SRBE_FLAG_NO_CP)
    refs = []
    for w, Q, seed in zip(ws, Qs, c["seeds"]):
        ks, _ = sampler.draw_kset(p, seed, 0, STEP)
        refs.append(dict(b=srbe.srbe_b(p, ks, w["ion_pos"], w["ion_q"], ele),
                         F=srbe.srbe_ion_forces(p, ks, w["ion_pos"], w["ion_q"], ele, Q), kset=ks))
    inputs = gpu_inputs([w["ion_pos"] for w in ws], [w["ion_q"] for w in ws], c["dpsi"], c["seeds"])
    qin = torch.tensor(np.concatenate(Qs), device="cuda")
    return dict(sys=sysm, refs=refs, inputs=inputs, qin=qin, n_ele=len(ele))


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request):
    c = build_case(request.param)
    c["name"] = request.param
    yield c
    c["sys"].close()


def check(case, precision, off, out, label):
    n = case["n_ele"]
    for r, ref in enumerate(case["refs"]):
        assert np.array_equal(out["kset"].cpu().numpy()[r * ref["kset"].size:(r + 1) * ref["kset"].size],
                              ref["kset"].astype(np.int32).ravel()), (label, r)
        F = forces_from_soa(out["F"], off, r)
        b = out["b"].cpu().numpy()[r * n:(r + 1) * n]
        print(f"{label} replica {r}: force {rel_rms(F, ref['F']):.2e} rms {rel_inf(F, ref['F']):.2e} max, "
              f"b {rel_rms(b, ref['b']):.2e} rms", flush=True)
        if precision == 0:
            assert rel_inf(F, ref["F"]) < 1e-11, (label, r)
            assert rel_inf(b, ref["b"]) < 1e-11, (label, r)
        else:
            assert rel_rms(F, ref["F"]) < 1e-5, (label, r)
            assert rel_rms(b, ref["b"]) < 3e-5, (label, r)


@pytest.mark.parametrize("precision", [0, 1])
def test_large_matches_oracle_and_graph_replay(case, precision):
    from paper_2509_24742_amd import binding
    off, xyz, q, dp, sd = case["inputs"]
    sysm = case["sys"]
    print(f"case {case['name']} precision {precision}: sizes {np.diff(off).tolist()} n_ele {case['n_ele']}",
          flush=True)
    out = sysm.step(off, xyz, q, dp, sd, STEP, precision=precision, Q_in=case["qin"])
    torch.cuda.synchronize()
    assert binding.srbe_sync_status(sysm.h) == 0, binding.srbe_last_error(sysm.h)
    check(case, precision, off, out, f"{case['name']} eager")
    gr = sysm.capture(off, xyz, q, dp, sd, STEP, precision=precision, Q_in=case["qin"])
    try:
        gr.launch()
        torch.cuda.synchronize()
        assert binding.srbe_sync_status(sysm.h) == 0, binding.srbe_last_error(sysm.h)
        for key in ("F", "b", "Q", "kset"):
            assert torch.equal(gr.out[key], out[key]), key
    finally:
        gr.close()


# ---------------------------------------------------------------- the full-size large slab

@pytest.fixture(scope="module")
def full():
    # 917,504 ions and 131,072 electrodes (2 x 256 x 256 walls) in 30 x 30 x 100 nm, M = 64,
    # P = 500, fixed charges; oracle values at 64 sampled ions and electrodes come from
    # tests/golden/large_slab_sample.json (written by make_large_slab_sample.py beside it)
    import json
    import os
    import sys
    import paper_2509_24742_amd as srbe_amd
    gdir = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    sys.path.insert(0, gdir)
    import make_large_slab_sample as golden
    with open(os.path.join(gdir, "large_slab_sample.json")) as f:
        ref = json.load(f)
    w, Q, ii, ie = golden.inputs()
    assert float(np.sum(w["ion_pos"] * np.arange(1, 4))) == ref["ion_pos_checksum"]
    assert ii.tolist() == ref["ion_index"] and ie.tolist() == ref["ele_index"]
    wp = dict(w["params"], kspace_tol=1e-16)
    sysm = srbe_amd.System(wp, w["ele_pos"], w["ele_side"], flags=srbe_amd.SRBE_FLAG_NO_CP)
    inputs = gpu_inputs([w["ion_pos"]], [w["ion_q"]], [w["dpsi"]], [ref["seed"]])
    yield dict(sys=sysm, ref=ref, inputs=inputs, qin=torch.tensor(Q, device="cuda"), p=oracle_params(wp),
               ii=ii, ie=ie, w=w)
    sysm.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_full_size_large_slab_at_sampled_targets(full, precision):
    from paper_2509_24742_amd import binding
    off, xyz, q, dp, sd = full["inputs"]
    ref = full["ref"]
    sysm = full["sys"]
    print(f"full-size large slab, precision {precision}: {ref['n_ion']} ions, {ref['n_ele']} electrodes", flush=True)
    out = sysm.step(off, xyz, q, dp, sd, ref["step"], precision=precision, Q_in=full["qin"])
    torch.cuda.synchronize()
    assert binding.srbe_sync_status(sysm.h) == 0, binding.srbe_last_error(sysm.h)
    ks, _ = sampler.draw_kset(full["p"], ref["seed"], 0, ref["step"])
    assert np.array_equal(out["kset"].cpu().numpy(), ks.astype(np.int32).ravel())
    F = forces_from_soa(out["F"], off, 0)[full["ii"]]
    b = out["b"].cpu().numpy()[full["ie"]]
    Fr, br = np.asarray(ref["F"]), np.asarray(ref["b"])
    print(f"  sampled force {rel_rms(F, Fr):.2e} rms {rel_inf(F, Fr):.2e} max, b {rel_rms(b, br):.2e} rms",
          flush=True)
    if precision == 0:
        assert rel_inf(F, Fr) < 1e-11 and rel_inf(b, br) < 1e-11
    else:
        assert rel_rms(F, Fr) < 1e-5 and rel_rms(b, br) < 3e-5


def test_full_size_large_slab_lattice_charge_solve(full):
    # the constant-potential step of the full-size slab with the lattice charge solve
    # (the dense S_ext would hold 131,072^2 doubles).  The ions' own induced charge
    # (~18 e per wall here) dwarfs what 2 V across 100 nm induces (~1 e), so the checks
    # are the voltage response: Q is neutral and exactly linear in dpsi (b* does not
    # depend on it), raising dpsi moves positive charge onto the positive wall, and
    # FP32 and FP64 agree to the FP32 path's error
    import paper_2509_24742_amd as srbe_amd
    from paper_2509_24742_amd import binding, workloads as wl
    off, xyz, q, dp, sd = full["inputs"]
    w = wl.large_slab()
    wp = dict(w["params"], kspace_tol=1e-16)
    side = np.asarray(w["ele_side"])
    sysm = srbe_amd.System(wp, w["ele_pos"], side, flags=srbe_amd.SRBE_FLAG_LATTICE_SOLVE)
    try:
        Q = {}
        for precision, dpsi in [(0, 0.0), (0, 2.0), (0, 4.0), (1, 2.0)]:
            dpt = torch.tensor([dpsi], dtype=torch.float64, device="cuda")
            out = sysm.step(off, xyz, q, dpt, sd, full["ref"]["step"], precision=precision)
            torch.cuda.synchronize()
            assert binding.srbe_sync_status(sysm.h) == 0, binding.srbe_last_error(sysm.h)
            Qv = out["Q"].cpu().numpy()
            print(f"  lattice solve, precision {precision}, dpsi {dpsi}: sum Q / sum |Q| = "
                  f"{np.sum(Qv) / np.sum(np.abs(Qv)):.2e}, wall charges {np.sum(Qv[side < 0]):.6f} "
                  f"{np.sum(Qv[side > 0]):.6f}, psibar {float(out['psibar'][0]):.6f}", flush=True)
            assert abs(np.sum(Qv)) < 1e-12 * np.sum(np.abs(Qv))
            assert np.isfinite(float(out["E"][0])) and np.isfinite(float(out["psibar"][0]))
            Q[(precision, dpsi)] = Qv
        # the response to 2 V is ~1/20 of Q, and Q a ~1e-6 remnant of b* (~400): the
        # difference of two FP64 solves carries ~1e-8 relative rounding
        d1 = Q[(0, 2.0)] - Q[(0, 0.0)]
        d2 = Q[(0, 4.0)] - Q[(0, 2.0)]
        e32 = rel_rms(Q[(1, 2.0)], Q[(0, 2.0)])
        print(f"  linearity {rel_inf(d2, d1):.2e}, FP32 vs FP64 charges {e32:.2e} rms", flush=True)
        assert rel_inf(d2, d1) < 1e-7
        assert np.sum(d1[side > 0]) > 0 > np.sum(d1[side < 0])
        assert e32 < 1e-4
    finally:
        sysm.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_full_size_large_slab_P2000_at_sampled_targets(full, precision):
    # the same slab, charges and sampled targets with a batch of P = 2000 modes
    # (tests/golden/large_slab_sample_P2000.json, written by make_large_slab_sample.py 2000)
    import json
    import os
    import paper_2509_24742_amd as srbe_amd
    from paper_2509_24742_amd import binding
    gdir = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    with open(os.path.join(gdir, "large_slab_sample_P2000.json")) as f:
        ref = json.load(f)
    assert ref["P"] == 2000 and ref["ion_index"] == full["ii"].tolist() and ref["ele_index"] == full["ie"].tolist()
    w = full["w"]
    wp = dict(w["params"], kspace_tol=1e-16, P=2000)
    sysm = srbe_amd.System(wp, w["ele_pos"], w["ele_side"], flags=srbe_amd.SRBE_FLAG_NO_CP)
    try:
        off, xyz, q, dp, sd = full["inputs"]
        sd = torch.tensor([ref["seed"]], dtype=torch.int64, device="cuda").view(torch.uint64)
        print(f"full-size large slab, P = 2000, precision {precision}", flush=True)
        out = sysm.step(off, xyz, q, dp, sd, ref["step"], precision=precision, Q_in=full["qin"])
        torch.cuda.synchronize()
        assert binding.srbe_sync_status(sysm.h) == 0, binding.srbe_last_error(sysm.h)
        ks, _ = sampler.draw_kset(oracle_params(wp), ref["seed"], 0, ref["step"])
        assert np.array_equal(out["kset"].cpu().numpy(), ks.astype(np.int32).ravel())
        F = forces_from_soa(out["F"], off, 0)[full["ii"]]
        b = out["b"].cpu().numpy()[full["ie"]]
        Fr, br = np.asarray(ref["F"]), np.asarray(ref["b"])
        print(f"  sampled force {rel_rms(F, Fr):.2e} rms {rel_inf(F, Fr):.2e} max, b {rel_rms(b, br):.2e} rms",
              flush=True)
        if precision == 0:
            assert rel_inf(F, Fr) < 1e-11 and rel_inf(b, br) < 1e-11
        else:
            assert rel_rms(F, Fr) < 1e-5 and rel_rms(b, br) < 3e-5
    finally:
        sysm.close()


# ---------------------------------------------------------------- the large-slab recipe at 1/8 scale

@pytest.fixture(scope="module")
def mid():
    # 2 x 32 x 32 square walls (2,048 atoms), 1,792 ions, 3.75 x 3.75 x 12.5 nm (aspect 10):
    # the constant-potential step by the lattice charge solve against the oracle's dense
    # solve (tests/golden/large_slab_mid.json, written by make_large_slab_mid.py beside it)
    import json
    import os
    import sys
    gdir = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    sys.path.insert(0, gdir)
    import make_large_slab_mid as golden
    with open(os.path.join(gdir, "large_slab_mid.json")) as f:
        ref = json.load(f)
    w, ii, ie = golden.inputs(500)
    assert float(np.sum(w["ion_pos"] * np.arange(1, 4))) == ref["ion_pos_checksum"]
    assert ii.tolist() == ref["ion_index"] and ie.tolist() == ref["ele_index"]
    yield dict(w=w, ref=ref, ii=ii, ie=ie)


@pytest.mark.parametrize("P", [500, 2000])
@pytest.mark.parametrize("precision", [0, 1])
def test_mid_size_slab_constant_potential_matches_oracle(mid, P, precision):
    import paper_2509_24742_amd as srbe_amd
    from paper_2509_24742_amd import binding
    w, ref = mid["w"], mid["ref"][str(P)]
    wp = dict(w["params"], kspace_tol=1e-16, P=P)
    sysm = srbe_amd.System(wp, w["ele_pos"], w["ele_side"], flags=srbe_amd.SRBE_FLAG_LATTICE_SOLVE)
    try:
        off, xyz, q, dp, sd = gpu_inputs([w["ion_pos"]], [w["ion_q"]], [w["dpsi"]], [mid["ref"]["seed"]])
        out = sysm.step(off, xyz, q, dp, sd, mid["ref"]["step"], precision=precision)
        torch.cuda.synchronize()
        assert binding.srbe_sync_status(sysm.h) == 0, binding.srbe_last_error(sysm.h)
        Q = out["Q"].cpu().numpy()
        F = forces_from_soa(out["F"], off, 0)[mid["ii"]]
        b = out["b"].cpu().numpy()[mid["ie"]]
        E, psibar = float(out["E"][0]), float(out["psibar"][0])
        Qr, Fr, br = np.asarray(ref["Q"]), np.asarray(ref["F"]), np.asarray(ref["b"])
        eE = abs(E - ref["E"]) / abs(ref["E"])
        print(f"mid-size slab P {P} precision {precision}: Q {rel_rms(Q, Qr):.2e} rms {rel_inf(Q, Qr):.2e} max, "
              f"F {rel_rms(F, Fr):.2e}, b {rel_rms(b, br):.2e}, E {eE:.2e}, psibar {abs(psibar - ref['psibar']):.2e}",
              flush=True)
        if precision == 0:
            assert rel_inf(Q, Qr) < 1e-10 and rel_inf(F, Fr) < 1e-11 and rel_inf(b, br) < 1e-11
            assert eE < 1e-11 and abs(psibar - ref["psibar"]) < 1e-11 * max(1.0, abs(ref["psibar"]))
        else:
            assert rel_rms(F, Fr) < 1e-5 and rel_rms(b, br) < 3e-5 and rel_rms(Q, Qr) < 1e-4
            assert abs(np.sum(Q)) < 1e-12 * np.sum(np.abs(Q))
    finally:
        sysm.close()
