"""srbe_step_noalloc (workspace in the library's fixed device scratch array) against srbe_step.

Both run the same kernels with the same launch parameters on the same inputs, and the
step is bitwise repeatable, so every output must be identical.  Two no-allocation calls
in a row on one handle, the second with fewer replicas and ions than the first (the
scratch keeps the first call's contents, which the second must not depend on), in FP64
and FP32, at constant potential and with fixed charges.  A step whose workspace exceeds
the scratch array is refused with SRBE_EINVAL before any device work.
"""

import numpy as np
import pytest

from helpers import gpu_inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def tiny():
    import paper_2509_24742_amd as srbe_amd
    from paper_2509_24742_amd import workloads as wl
    ws = [wl.tiny_slab(seed=1000 + r) for r in range(4)]
    wp = dict(ws[0]["params"], kspace_tol=1e-16)
    sysm = srbe_amd.System(wp, ws[0]["ele_pos"], ws[0]["ele_side"])
    yield dict(ws=ws, sys=sysm)
    sysm.close()


def _outputs(sysm, off, dev):
    return sysm.outputs(off, dev)


def _run(sysm, entry, off, xyz, q, dp, sd, step, precision, Q_in=None):
    out = _outputs(sysm, off, dp.device)
    for v in out.values():
        if v is not None:
            v.fill_(float("nan")) if v.is_floating_point() else v.fill_(-7)
    entry(sysm.h, precision, off, xyz, q, dp, sd, step, out["Q"], out["F"], Q_in=Q_in, b_out=out["b"],
          psibar_out=out["psibar"], energy_out=out["E"], kset_out=out["kset"])
    torch.cuda.synchronize()
    from paper_2509_24742_amd import binding
    assert binding.srbe_sync_status(sysm.h) == 0, binding.srbe_last_error(sysm.h)
    return {k: v.cpu().numpy() for k, v in out.items() if v is not None}


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("fixed", [False, True])
def test_noalloc_equals_step_twice_shrinking(tiny, precision, fixed):
    from paper_2509_24742_amd import binding
    ws, sysm = tiny["ws"], tiny["sys"]
    for nrep, step in ((4, 5), (2, 6)):
        reps = ws[:nrep]
        # the second call also drops ions from its last replica (a smaller, ragged batch)
        pos = [w["ion_pos"] for w in reps]
        qs = [w["ion_q"] for w in reps]
        if nrep == 2:
            pos[-1], qs[-1] = pos[-1][:150], qs[-1][:150]
            qs[-1] = qs[-1] - qs[-1].mean()  # keep the replica neutral
        off, xyz, q, dp, sd = gpu_inputs(pos, qs, [2.0 - 0.5 * r for r in range(nrep)],
                                         [3000 + r for r in range(nrep)])
        Q_in = None
        if fixed:
            Q_in = torch.tensor(np.random.default_rng(nrep).normal(size=nrep * sysm.n_ele) * 0.01,
                                dtype=torch.float64, device=dp.device)
        print(f"precision {precision} fixed {fixed}: {nrep} replicas, {int(off[-1])} ions", flush=True)
        ref = _run(sysm, binding.srbe_step, off, xyz, q, dp, sd, step, precision, Q_in)
        got = _run(sysm, binding.srbe_step_noalloc, off, xyz, q, dp, sd, step, precision, Q_in)
        for key in ref:
            assert np.array_equal(got[key], ref[key], equal_nan=True), key
        assert np.all(np.isfinite(got["F"])) and np.all(np.isfinite(got["Q"]))


def test_noalloc_refuses_a_workspace_beyond_the_scratch(tiny):
    from paper_2509_24742_amd import binding
    sysm = tiny["sys"]
    n = 1 << 20  # ~100 bytes of workspace per ion: beyond the 64 MiB array
    off = np.array([0, n], dtype=np.int64)
    dev = torch.device("cuda")
    xyz = torch.zeros(3 * n, dtype=torch.float64, device=dev)
    q = torch.zeros(n, dtype=torch.float64, device=dev)
    dp = torch.zeros(1, dtype=torch.float64, device=dev)
    sd = torch.zeros(1, dtype=torch.int64, device=dev).view(torch.uint64)
    out = sysm.outputs(off, dev)
    code = binding.srbe_step_noalloc(sysm.h, 1, off, xyz, q, dp, sd, 0, out["Q"], out["F"], check=False)
    assert code == binding.SRBE_EINVAL
    assert "scratch" in binding.srbe_last_error(sysm.h)
