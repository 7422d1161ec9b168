"""The electrostatic virial tensor (srbe_virial) against ``oracle.virial.srbe_virial``.

The oracle's virial is pinned on the CPU (finite differences of the strained energy,
the Coulomb trace identity, the exact expectation over every mode).  Here the library's
tensor after a constant-potential step is compared with the oracle's at the oracle's
own charges and the same sample: two replicas of the tiny slab (rc = 1.19 nm, off the
walls' 1.2 nm site distances, where the two sides may decide a pair differently), FP64
to 1e-11 of the largest component, FP32 to 2e-6 of it (measured ~1e-7: the Fourier part
comes from the FP32 structure factors, the rest is FP64), every component.
"""

import numpy as np
import pytest

from helpers import gpu_inputs, oracle_params, oracle_solver, oracle_step

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("precision", [0, 1])
def test_virial_matches_oracle(precision):
    import paper_2509_24742_amd as srbe_amd
    from oracle import virial
    from paper_2509_24742_amd import binding
    from paper_2509_24742_amd import workloads as wl
    w = wl.tiny_slab()
    w2 = wl.tiny_slab(seed=8)
    wp = dict(w["params"], kspace_tol=1e-16, rc=1.19)
    p = oracle_params(wp)
    solver = oracle_solver(p, w["ele_pos"])
    ions, qs, dps, seeds = [w["ion_pos"], w2["ion_pos"]], [w["ion_q"], w2["ion_q"]], [w["dpsi"], 0.7], [31, 32]
    sysm = srbe_amd.System(wp, w["ele_pos"], w["ele_side"])
    try:
        off, xyz, q, dp, sd = gpu_inputs(ions, qs, dps, seeds)
        out = sysm.step(off, xyz, q, dp, sd, 4, precision=precision)  # its Q_out is read by srbe_virial
        W = torch.empty(12, dtype=torch.float64, device="cuda")
        binding.srbe_virial(sysm.h, 2, W)
        torch.cuda.synchronize()
        assert binding.srbe_sync_status(sysm.h) == 0, binding.srbe_last_error(sysm.h)
        got = W.cpu().numpy().reshape(2, 6)
        del out
        for r in range(2):
            ref = oracle_step(p, solver, seeds[r], 4, ions[r], qs[r], w["ele_pos"], w["ele_side"], dps[r])
            Wr = virial.srbe_virial(p, ref["kset"], ions[r], qs[r], w["ele_pos"], ref["Q"])
            err = np.max(np.abs(got[r] - Wr)) / np.max(np.abs(Wr))
            print(f"precision {precision} replica {r}: W {np.array2string(Wr, precision=4)} got "
                  f"{np.array2string(got[r], precision=4)} err {err:.2e}", flush=True)
            assert err < (1e-11 if precision == 0 else 2e-6)
    finally:
        sysm.close()


def test_virial_needs_a_step():
    import paper_2509_24742_amd as srbe_amd
    from paper_2509_24742_amd import binding
    from paper_2509_24742_amd import workloads as wl
    w = wl.tiny_slab()
    sysm = srbe_amd.System(dict(w["params"], kspace_tol=1e-16), w["ele_pos"], w["ele_side"])
    try:
        with pytest.raises(binding.SrbeError):
            binding.srbe_virial(sysm.h, 1, torch.empty(6, dtype=torch.float64, device="cuda"))
    finally:
        sysm.close()
