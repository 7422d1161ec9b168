"""Captured steps (srbe_graph_*): every replay equals the eager step with the same
step index, bit for bit.  Replays are interleaved with eager steps and host
synchronisations, and the step counter is advanced by the replays and reset by
srbe_graph_set_step."""

import numpy as np
import pytest

from helpers import gpu_inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _replicas(R):
    from paper_2509_24742_amd import workloads as wl
    rng = np.random.default_rng(77)
    w = wl.tiny_slab()
    p = w["params"]
    reps = []
    for r in range(R):
        pos = wl.jitter(w["ion_pos"], 0.02, rng, p["Lx"], p["Ly"], 0.3, p["H"] - 0.3)
        reps.append((pos, w["ion_q"]))
    return w, reps


def _same(a, b):
    for k in ("Q", "F", "b", "psibar", "E", "kset"):
        if a[k] is None:
            continue
        x, y = a[k].cpu().numpy(), b[k].cpu().numpy()
        assert np.array_equal(x.view(np.uint8), y.view(np.uint8)), k


@pytest.mark.parametrize("precision", [0, 1])
def test_graph_replays_match_eager(precision):
    import paper_2509_24742_amd as srbe_amd
    from paper_2509_24742_amd import binding
    R = 3
    w, reps = _replicas(R)
    sysm = srbe_amd.System(dict(w["params"], kspace_tol=1e-16), w["ele_pos"], w["ele_side"])
    off, xyz, q, dp, sd = gpu_inputs([r[0] for r in reps], [r[1] for r in reps], [0.5, 1.0, 2.0], [11, 12, 13])
    first = 40
    gr = sysm.capture(off, xyz, q, dp, sd, first, precision=precision)
    try:
        for i in range(4):
            out_g = gr.launch()
            torch.cuda.synchronize()
            assert binding.srbe_sync_status(sysm.h) == 0, binding.srbe_last_error(sysm.h)
            got = {k: (v.clone() if v is not None else None) for k, v in out_g.items()}
            ref = sysm.step(off, xyz, q, dp, sd, first + i, precision=precision)  # eager work between replays
            torch.cuda.synchronize()
            _same(got, ref)
        gr.set_step(first + 1)
        out_g = gr.launch()
        torch.cuda.synchronize()
        got = {k: (v.clone() if v is not None else None) for k, v in out_g.items()}
        ref = sysm.step(off, xyz, q, dp, sd, first + 1, precision=precision)
        torch.cuda.synchronize()
        _same(got, ref)
    finally:
        gr.close()
        sysm.close()


def test_graph_fixed_charges():
    import paper_2509_24742_amd as srbe_amd
    w, reps = _replicas(2)
    sysm = srbe_amd.System(dict(w["params"], kspace_tol=1e-16), w["ele_pos"], w["ele_side"])
    off, xyz, q, dp, sd = gpu_inputs([r[0] for r in reps], [r[1] for r in reps], [1.0, 2.0], [5, 6])
    Qin = torch.tensor(np.random.default_rng(3).normal(scale=1e-3, size=2 * sysm.n_ele), dtype=torch.float64,
                       device="cuda")
    gr = sysm.capture(off, xyz, q, dp, sd, 7, precision=1, Q_in=Qin)
    try:
        out_g = gr.launch()
        torch.cuda.synchronize()
        got = {k: (v.clone() if v is not None else None) for k, v in out_g.items()}
        ref = sysm.step(off, xyz, q, dp, sd, 7, precision=1, Q_in=Qin)
        torch.cuda.synchronize()
        _same(got, ref)
    finally:
        gr.close()
        sysm.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_split_launches_match_fused(precision):
    """With phase timing on, the fused launches run part by part; the results are the
    same bits as the fused step's."""
    import paper_2509_24742_amd as srbe_amd
    from paper_2509_24742_amd import binding
    R = 3
    w, reps = _replicas(R)
    sysm = srbe_amd.System(dict(w["params"], kspace_tol=1e-16), w["ele_pos"], w["ele_side"])
    off, xyz, q, dp, sd = gpu_inputs([r[0] for r in reps], [r[1] for r in reps], [0.5, 1.0, 2.0], [21, 22, 23])
    try:
        ref = sysm.step(off, xyz, q, dp, sd, 9, precision=precision)
        torch.cuda.synchronize()
        ref = {k: (v.clone() if v is not None else None) for k, v in ref.items()}
        binding.srbe_profile_enable(sysm.h, True)
        got = sysm.step(off, xyz, q, dp, sd, 9, precision=precision)
        torch.cuda.synchronize()
        prof = binding.srbe_profile_read(sysm.h)
        binding.srbe_profile_enable(sysm.h, False)
        assert binding.srbe_sync_status(sysm.h) == 0, binding.srbe_last_error(sysm.h)
        _same(got, ref)
        for name in ("sample", "cellsort", "sf_ions", "real_ele", "real_ii", "ele_potential", "cp_gemm",
                     "post_charges", "sf_ele", "real_ie", "ion_force", "energy", "sf_ions_finalize",
                     "sf_ele_finalize"):
            assert prof[name][1] == 1, (name, prof[name])
    finally:
        sysm.close()
