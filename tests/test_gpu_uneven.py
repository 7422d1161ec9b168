"""Systems of the uneven batch (32 slabs of 2e3-2e5 particles, each its own box).

Every system has two square-lattice walls, so each runs on its own handle with the
lattice charge solve (SRBE_FLAG_LATTICE_SOLVE), and the large ones take the
multi-block cell sort.  The three smallest systems (2,108, 2,614 and 2,718
particles; aspect ratios 12, 4.5 and 12) are compared in full with the FP64 oracle,
whose charges come from its dense solve, to the tolerances of test_gpu_step.py
(FP64: 1e-11 relative max-norm; FP32: force relative RMS <= 1e-5, b and Q <= 3e-5).
The oracle's electrode matrix for the larger systems would take hours; their
kernels are the ones the large-replica and lattice tests check.
"""

import numpy as np
import pytest

from helpers import forces_from_soa, gpu_inputs, oracle_params, oracle_solver, oracle_step, rel_inf, rel_rms

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SMALLEST = [10, 16, 7]
STEP = 2


@pytest.fixture(scope="module", params=SMALLEST)
def system(request):
    import paper_2509_24742_amd as srbe_amd
    from paper_2509_24742_amd import workloads as wl
    w = wl.uneven_batch(place={request.param})[request.param]
    wp = dict(w["params"], kspace_tol=1e-16)
    p = oracle_params(wp)
    solver = oracle_solver(p, w["ele_pos"])
    seed = 4100 + request.param
    ref = oracle_step(p, solver, seed, STEP, w["ion_pos"], w["ion_q"], w["ele_pos"], w["ele_side"], w["dpsi"])
    sysm = srbe_amd.System(wp, w["ele_pos"], w["ele_side"], flags=srbe_amd.SRBE_FLAG_LATTICE_SOLVE)
    inputs = gpu_inputs([w["ion_pos"]], [w["ion_q"]], [w["dpsi"]], [seed])
    yield dict(sys=sysm, ref=ref, inputs=inputs, n=len(w["ele_side"]), k=request.param, N=w["n_total"])
    sysm.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_uneven_system_matches_oracle(system, precision):
    from paper_2509_24742_amd import binding
    off, xyz, q, dp, sd = system["inputs"]
    out = system["sys"].step(off, xyz, q, dp, sd, STEP, precision=precision)
    torch.cuda.synchronize()
    assert binding.srbe_sync_status(system["sys"].h) == 0, binding.srbe_last_error(system["sys"].h)
    ref = system["ref"]
    F = forces_from_soa(out["F"], off, 0)
    b, Q = out["b"].cpu().numpy(), out["Q"].cpu().numpy()
    E = float(out["E"][0])
    print(f"system {system['k']} ({system['N']} particles) precision {precision}: Q {rel_inf(Q, ref['Q']):.2e} max, "
          f"F {rel_rms(F, ref['F']):.2e} rms, b {rel_rms(b, ref['b']):.2e} rms, "
          f"E {abs(E - ref['E']) / abs(ref['E']):.2e}", flush=True)
    assert np.array_equal(out["kset"].cpu().numpy(), ref["kset"].astype(np.int32).ravel())
    if precision == 0:
        assert rel_inf(Q, ref["Q"]) < 1e-11 and rel_inf(b, ref["b"]) < 1e-11 and rel_inf(F, ref["F"]) < 1e-11
        assert abs(E - ref["E"]) < 1e-11 * abs(ref["E"])
    else:
        assert rel_rms(F, ref["F"]) < 1e-5
        assert rel_rms(b, ref["b"]) < 3e-5 and rel_rms(Q, ref["Q"]) < 3e-5


@pytest.mark.parametrize("precision", [0, 1])
def test_largest_uneven_system_at_sampled_targets(precision):
    # the largest system (162,990 particles: multi-block cell sort) at fixed charges against
    # the oracle at 64 sampled ions and electrodes (tests/golden/uneven_largest.json,
    # written by make_uneven_largest.py beside it)
    import json
    import os
    import sys
    import paper_2509_24742_amd as srbe_amd
    from paper_2509_24742_amd import binding
    gdir = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    sys.path.insert(0, gdir)
    import make_uneven_largest as golden
    with open(os.path.join(gdir, "uneven_largest.json")) as f:
        ref = json.load(f)
    w, Q, ii, ie = golden.inputs()
    assert float(np.sum(w["ion_pos"] * np.arange(1, 4))) == ref["ion_pos_checksum"]
    wp = dict(w["params"], kspace_tol=1e-16)
    sysm = srbe_amd.System(wp, w["ele_pos"], w["ele_side"], flags=srbe_amd.SRBE_FLAG_NO_CP)
    try:
        off, xyz, q, dp, sd = gpu_inputs([w["ion_pos"]], [w["ion_q"]], [w["dpsi"]], [ref["seed"]])
        out = sysm.step(off, xyz, q, dp, sd, ref["step"], precision=precision,
                        Q_in=torch.tensor(Q, dtype=torch.float64, device="cuda"))
        torch.cuda.synchronize()
        assert binding.srbe_sync_status(sysm.h) == 0, binding.srbe_last_error(sysm.h)
        F = forces_from_soa(out["F"], off, 0)[ii]
        b = out["b"].cpu().numpy()[ie]
        Fr, br = np.asarray(ref["F"]), np.asarray(ref["b"])
        print(f"largest uneven system precision {precision}: F {rel_rms(F, Fr):.2e} rms {rel_inf(F, Fr):.2e} max, "
              f"b {rel_rms(b, br):.2e}", flush=True)
        if precision == 0:
            assert rel_inf(F, Fr) < 1e-11 and rel_inf(b, br) < 1e-11
        else:
            assert rel_rms(F, Fr) < 1e-5 and rel_rms(b, br) < 3e-5
    finally:
        sysm.close()
