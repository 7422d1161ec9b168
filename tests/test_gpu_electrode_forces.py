"""Forces on the electrode atoms (srbe_electrode_forces) against the oracle.

After a step of three replicas of the tiny slab (the charge solve included), the
electrode forces are compared with the oracle's (``srbe.srbe_ele_forces``: the Fourier
force with S = S1 + S2, the slab force, and the real-space forces from the ions and
the other electrodes) at the oracle's charges and the same sample, to the tolerances of
test_gpu_step.py (FP64 1e-11 relative max-norm; FP32 relative RMS 1e-5).  The
momentum balance of a sample, sum over ions and electrodes of the force = 0, is checked
on the device's own FP64 forces.  Without a preceding step the call is refused.

The tiny slab runs with rc = 1.19 nm here: its walls' sites lie exactly 1.2 nm (six
spacings) apart, and for such pairs the device's rounded fractional differences and the
oracle's rounded coordinate differences can fall on opposite sides of the cutoff (the
kernel there is ~1e-7 of the force).
"""

import numpy as np
import pytest

from helpers import forces_from_soa, gpu_inputs, oracle_params, oracle_solver, oracle_step, rel_inf, rel_rms

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SEEDS = [2000, 31, 77]
DPSI = [2.0, 0.5, 3.0]
STEP = 6


@pytest.fixture(scope="module")
def tiny():
    import paper_2509_24742_amd as srbe_amd
    from paper_2509_24742_amd import workloads as wl
    w = wl.tiny_slab()
    w["params"] = dict(w["params"], rc=1.19)
    wp = dict(w["params"], kspace_tol=1e-16)
    p = oracle_params(wp)
    solver = oracle_solver(p, w["ele_pos"])
    sysm = srbe_amd.System(wp, w["ele_pos"], w["ele_side"])
    yield dict(w=w, p=p, solver=solver, sys=sysm)
    sysm.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_electrode_forces_match_oracle_and_balance_momentum(tiny, precision):
    from oracle import srbe
    from paper_2509_24742_amd import binding
    w, p, sysm = tiny["w"], tiny["p"], tiny["sys"]
    ion, q, ele = np.asarray(w["ion_pos"]), np.asarray(w["ion_q"]), np.asarray(w["ele_pos"])
    off, xyz, qt, dp, sd = gpu_inputs([ion] * 3, [q] * 3, DPSI, SEEDS)
    out = sysm.step(off, xyz, qt, dp, sd, STEP, precision=precision)
    n = len(ele)
    Fe = torch.empty(3 * 3 * n, dtype=torch.float64, device="cuda")
    binding.srbe_electrode_forces(sysm.h, 3, Fe)
    torch.cuda.synchronize()
    assert binding.srbe_sync_status(sysm.h) == 0, binding.srbe_last_error(sysm.h)
    Fe = Fe.cpu().numpy().reshape(3, 3 * n)
    Fi = out["F"].cpu().numpy().reshape(3, -1)
    for r, (seed, dpsi) in enumerate(zip(SEEDS, DPSI)):
        ref = oracle_step(p, tiny["solver"], seed, STEP, ion, q, ele, w["ele_side"], dpsi)
        Fref = srbe.srbe_ele_forces(p, ref["kset"], ion, q, ele, ref["Q"])
        got = Fe[:, r * n:(r + 1) * n].T
        print(f"precision {precision} replica {r}: electrode force {rel_rms(got, Fref):.2e} rms "
              f"{rel_inf(got, Fref):.2e} max", flush=True)
        if precision == 0:
            assert rel_inf(got, Fref) < 1e-11, r
            total = got.sum(axis=0) + Fi[:, off[r]:off[r + 1]].T.sum(axis=0)
            scale = max(np.abs(got).max(), np.abs(Fi).max())
            print(f"  momentum balance {np.abs(total).max() / scale:.2e}", flush=True)
            assert np.abs(total).max() < 1e-11 * scale, r
        else:
            assert rel_rms(got, Fref) < 1e-5, r


def test_electrode_forces_need_a_step(tiny):
    import paper_2509_24742_amd as srbe_amd
    from paper_2509_24742_amd import binding
    w = tiny["w"]
    fresh = srbe_amd.System(dict(w["params"], kspace_tol=1e-16), w["ele_pos"], w["ele_side"],
                            flags=srbe_amd.SRBE_FLAG_NO_CP)
    try:
        Fe = torch.empty(3 * fresh.n_ele, dtype=torch.float64, device="cuda")
        with pytest.raises(binding.SrbeError) as ei:
            binding.srbe_electrode_forces(fresh.h, 1, Fe)
        assert ei.value.code == binding.SRBE_EINVAL
    finally:
        fresh.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_electrode_forces_with_a_replica_without_ions(tiny, precision):
    """A batch whose middle replica has no ions (in FP32 its electrode records come from
    the ion-force launch's first block of that replica, which has no ions to move)."""
    from oracle import srbe
    from paper_2509_24742_amd import binding
    w, p, sysm = tiny["w"], tiny["p"], tiny["sys"]
    ion, q, ele = np.asarray(w["ion_pos"]), np.asarray(w["ion_q"]), np.asarray(w["ele_pos"])
    none_xyz, none_q = np.zeros((0, 3)), np.zeros(0)
    ions, qs = [ion, none_xyz, ion], [q, none_q, q]
    off, xyz, qt, dp, sd = gpu_inputs(ions, qs, DPSI, SEEDS)
    # the call reads the step's charges from its output buffers: `out` keeps them alive
    out = sysm.step(off, xyz, qt, dp, sd, STEP, precision=precision)
    n = len(ele)
    Fe = torch.empty(3 * 3 * n, dtype=torch.float64, device="cuda")
    binding.srbe_electrode_forces(sysm.h, 3, Fe)
    torch.cuda.synchronize()
    assert binding.srbe_sync_status(sysm.h) == 0, binding.srbe_last_error(sysm.h)
    Fe = Fe.cpu().numpy().reshape(3, 3 * n)
    err = []
    for r, (seed, dpsi) in enumerate(zip(SEEDS, DPSI)):
        ref = oracle_step(p, tiny["solver"], seed, STEP, ions[r], qs[r], ele, w["ele_side"], dpsi)
        Fref = srbe.srbe_ele_forces(p, ref["kset"], ions[r], qs[r], ele, ref["Q"])
        got = Fe[:, r * n:(r + 1) * n].T
        err.append(rel_rms(got, Fref))
        Qg = out["Q"].cpu().numpy()[r * n:(r + 1) * n]
        print(f"  Q {rel_rms(Qg, ref['Q']):.2e}", flush=True)
        if len(qs[r]):
            print(f"  F {rel_rms(forces_from_soa(out['F'], off, r), ref['F']):.2e}", flush=True)
        print(f"precision {precision} replica {r} ({len(qs[r])} ions): electrode force {err[-1]:.2e} rms", flush=True)
    assert max(err) < (1e-11 if precision == 0 else 1e-5), err
