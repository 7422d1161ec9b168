"""Edge cases of the GPU step against the oracle: a replica with no ions inside a
batch, a step with no ions at all (the empty capacitor), ions exactly on the walls
(z = 0 and z = H, the ends of the accepted range), and the two sides of the cell
sort's switch: the largest replica the one-block sort takes (8192 ions) and the
smallest the multi-block sort takes (8194 ions, ~100 per cell), both placed at
random, so close pairs occur.  Tolerances as in test_gpu_step.py.
"""

import numpy as np
import pytest

from helpers import forces_from_soa, gpu_inputs, oracle_params, oracle_solver, oracle_step, rel_inf, rel_rms

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def tiny():
    import paper_2509_24742_amd as srbe_amd
    from paper_2509_24742_amd import workloads as wl
    w = wl.tiny_slab()
    wp = dict(w["params"], kspace_tol=1e-16)
    p = oracle_params(wp)
    solver = oracle_solver(p, w["ele_pos"])
    sysm = srbe_amd.System(wp, w["ele_pos"], w["ele_side"])
    yield dict(w=w, wp=wp, p=p, solver=solver, sys=sysm)
    sysm.close()


def _run(tiny, reps, dpsi, seeds, step, prec):
    from paper_2509_24742_amd import binding
    off, xyz, q, dp, sd = gpu_inputs([r[0] for r in reps], [r[1] for r in reps], dpsi, seeds)
    out = tiny["sys"].step(off, xyz, q, dp, sd, step, precision=prec)
    torch.cuda.synchronize()
    assert binding.srbe_sync_status(tiny["sys"].h) == 0, binding.srbe_last_error(tiny["sys"].h)
    return off, out


def _check(tiny, reps, dpsi, seeds, step, prec, off, out):
    w = tiny["w"]
    n = len(w["ele_pos"])
    for r in range(len(reps)):
        ref = oracle_step(tiny["p"], tiny["solver"], seeds[r], step, reps[r][0], reps[r][1], w["ele_pos"],
                          w["ele_side"], dpsi[r])
        Qg = out["Q"].cpu().numpy()[r * n:(r + 1) * n]
        E = float(out["E"][r])
        if prec == 0:
            assert rel_inf(Qg, ref["Q"]) < 1e-11, r
            assert abs(E - ref["E"]) < 1e-11 * max(abs(ref["E"]), 1e-3), r
        else:
            assert rel_rms(Qg, ref["Q"]) < 3e-5, r
        if len(reps[r][1]):
            Fg = forces_from_soa(out["F"], off, r)
            if prec == 0:
                assert rel_inf(Fg, ref["F"]) < 1e-11, r
            else:
                assert rel_rms(Fg, ref["F"]) < 1e-5, r


@pytest.mark.parametrize("prec", [0, 1])
def test_replica_without_ions_in_a_batch(tiny, prec):
    w = tiny["w"]
    reps = [(w["ion_pos"], w["ion_q"]), (np.zeros((0, 3)), np.zeros(0)), (w["ion_pos"][:64], w["ion_q"][:64])]
    reps[2] = (np.concatenate([w["ion_pos"][:32], w["ion_pos"][100:132]]),
               np.concatenate([w["ion_q"][:32], w["ion_q"][100:132]]))
    dpsi, seeds = [1.0, 2.0, 0.5], [41, 42, 43]
    off, out = _run(tiny, reps, dpsi, seeds, 4, prec)
    _check(tiny, reps, dpsi, seeds, 4, prec, off, out)


def test_no_ions_at_all(tiny):
    # the empty capacitor: only the electrodes and the applied voltage remain
    reps = [(np.zeros((0, 3)), np.zeros(0))]
    off, out = _run(tiny, reps, [2.0], [7], 1, 0)
    _check(tiny, reps, [2.0], [7], 1, 0, off, out)


@pytest.mark.parametrize("prec", [0, 1])
def test_ions_on_the_walls(tiny, prec):
    w = tiny["w"]
    pos = w["ion_pos"].copy()
    pos[0, 2] = 0.0
    pos[1, 2] = w["params"]["H"]
    off, out = _run(tiny, [(pos, w["ion_q"])], [1.0], [9], 2, prec)
    _check(tiny, [(pos, w["ion_q"])], [1.0], [9], 2, prec, off, out)


@pytest.mark.parametrize("n", [8192, 8194])
@pytest.mark.parametrize("prec", [0, 1])
def test_replicas_at_the_sort_switch(tiny, prec, n):
    wp = tiny["wp"]
    rng = np.random.default_rng(5)
    pos = np.stack([rng.uniform(0, wp["Lx"], n), rng.uniform(0, wp["Ly"], n), rng.uniform(0.2, wp["H"] - 0.2, n)], 1)
    q = np.where(np.arange(n) % 2 == 0, 0.5, -0.5)
    print(f"replica of {n} ions, precision {prec}", flush=True)
    off, out = _run(tiny, [(pos, q)], [1.0], [17], 3, prec)
    _check(tiny, [(pos, q)], [1.0], [17], 3, prec, off, out)
