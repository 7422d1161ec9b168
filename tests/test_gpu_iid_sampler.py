"""The i.i.d. sampler option (SRBE_FLAG_IID_SAMPLER) against ``oracle.sampler.iid_draw_kset``.

Rejection sampling with the Metropolis sampler's proposal and target (pinned on the CPU
by a chi^2 test of its counts and by its exact acceptance rate).  On the GPU: the modes
and the attempt counts equal the oracle's bit for bit (three seeds, three steps; P = 100
on the tiny slab, one round of 1024 attempts, and P = 2000 on the paper-shaped cell,
three rounds), and a whole constant-potential step drawn this way matches the oracle's
step on the same sample to 1e-11 (FP64).
"""

import numpy as np
import pytest

from helpers import forces_from_soa, gpu_inputs, oracle_params, oracle_solver, oracle_step, rel_inf

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("cell,P", [("tiny", 100), ("paper", 2000)])
def test_iid_sample_bit_exact(cell, P):
    import paper_2509_24742_amd as srbe_amd
    from oracle import sampler
    from paper_2509_24742_amd import workloads as wl
    w = wl.tiny_slab() if cell == "tiny" else wl.paper_cell()
    wp = dict(w["params"], kspace_tol=1e-16, P=P)
    p = oracle_params(wp)
    sysm = srbe_amd.System(wp, w["ele_pos"], w["ele_side"],
                           flags=srbe_amd.SRBE_FLAG_IID_SAMPLER | srbe_amd.SRBE_FLAG_NO_CP)
    try:
        seeds = np.array([2000, 7, 2 ** 40 + 3], dtype=np.uint64)
        sd = torch.tensor(seeds.view(np.int64), device="cuda").view(torch.uint64)
        for step in (0, 1, 12345):
            ks = torch.empty(len(seeds) * P * 3, dtype=torch.int32, device="cuda")
            natt = torch.empty(len(seeds), dtype=torch.int32, device="cuda")
            srbe_amd.srbe_sample(sysm.h, sd, step, ks, natt)
            got = ks.cpu().numpy().reshape(len(seeds), P, 3)
            for r, s in enumerate(seeds):
                ref, att = sampler.iid_draw_kset(p, int(s), 0, step)
                assert np.array_equal(got[r], ref), f"seed {s} step {step}"
                assert int(natt[r]) == att
                assert att < 65536
        print(f"{cell} P={P}: acceptance {P / att:.3f}", flush=True)
    finally:
        sysm.close()


def test_iid_step_matches_oracle():
    import paper_2509_24742_amd as srbe_amd
    from oracle import sampler
    from paper_2509_24742_amd import binding
    from paper_2509_24742_amd import workloads as wl
    w = wl.tiny_slab()
    wp = dict(w["params"], kspace_tol=1e-16)
    p = oracle_params(wp)
    sysm = srbe_amd.System(wp, w["ele_pos"], w["ele_side"], flags=srbe_amd.SRBE_FLAG_IID_SAMPLER)
    try:
        off, xyz, q, dp, sd = gpu_inputs([w["ion_pos"]], [w["ion_q"]], [w["dpsi"]], [77])
        out = sysm.step(off, xyz, q, dp, sd, 9, precision=0)
        torch.cuda.synchronize()
        assert binding.srbe_sync_status(sysm.h) == 0, binding.srbe_last_error(sysm.h)
        ks, _ = sampler.iid_draw_kset(p, 77, 0, 9)
        ref = oracle_step(p, oracle_solver(p, w["ele_pos"]), 77, 9, w["ion_pos"], w["ion_q"], w["ele_pos"],
                          w["ele_side"], w["dpsi"], kset=ks)
        assert np.array_equal(out["kset"].cpu().numpy(), ks.astype(np.int32).ravel())
        F = forces_from_soa(out["F"], off, 0)
        assert rel_inf(F, ref["F"]) < 1e-11
        assert rel_inf(out["Q"].cpu().numpy(), ref["Q"]) < 1e-11
        assert abs(float(out["E"][0]) - ref["E"]) < 1e-11 * abs(ref["E"])
    finally:
        sysm.close()
