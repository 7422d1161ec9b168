"""Parity at the benchmark's full size and launch configuration: the 64-replica batch
of paper-shaped cells (1280 ion sites + 2160 electrode atoms each, M = 13, P = 200),
FP32 path, one replay of a captured step, against the FP64 oracle on sampled
replicas with the same k-sets; and the FP64 path on one paper-shaped cell.

Tolerances as in test_gpu_step.py (derived there): FP32 force relative RMS <= 1e-5
(the stated target), b and Q <= 3e-5 relative RMS, energy <= 1e-6 of the scale of
its terms; FP64 <= 1e-11 relative in the max norm (Q: 1e-10, the condition number
of A being ~1e4 for the 2160-atom electrodes).  The oracle's electrode matrix is
built once (about half a minute on 16 threads).
"""

import numpy as np
import pytest

from helpers import energy_scale, forces_from_soa, oracle_params, oracle_solver, oracle_step, rel_inf, rel_rms

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SAMPLED = (0, 29, 63)


@pytest.fixture(scope="module")
def batch():
    import paper_2509_24742_amd as srbe_amd
    from paper_2509_24742_amd import workloads as wl
    wb = wl.replica_batch(R=64)
    wp = dict(wb["params"], kspace_tol=1e-16)
    p = oracle_params(wp)
    print("building the oracle's electrode matrix", flush=True)
    solver = oracle_solver(p, wb["ele_pos"])
    sysm = srbe_amd.System(wp, wb["ele_pos"], wb["ele_side"])
    yield dict(wb=wb, wp=wp, p=p, solver=solver, sys=sysm)
    sysm.close()


def _inputs(wb, reps, seeds):
    dev = torch.device("cuda:0")
    sizes = [len(wb["ion_q"][r]) for r in reps]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    pos = np.concatenate([wb["ion_pos"][r] for r in reps])
    xyz = torch.tensor(np.ascontiguousarray(pos.T).ravel(), dtype=torch.float64, device=dev)
    q = torch.tensor(np.concatenate([wb["ion_q"][r] for r in reps]), dtype=torch.float64, device=dev)
    dp = torch.tensor(np.asarray(wb["dpsi"])[list(reps)], dtype=torch.float64, device=dev)
    sd = torch.tensor(np.asarray(seeds, dtype=np.int64), dtype=torch.int64, device=dev).view(torch.uint64)
    return off, xyz, q, dp, sd


def test_fp32_graph_replay_full_batch(batch):
    from paper_2509_24742_amd import binding
    wb, p, sysm = batch["wb"], batch["p"], batch["sys"]
    R = 64
    seeds = 2100 + np.arange(R)
    off, xyz, q, dp, sd = _inputs(wb, range(R), seeds)
    step = 3
    gr = sysm.capture(off, xyz, q, dp, sd, step, precision=1)
    try:
        out = gr.launch()
        torch.cuda.synchronize()
        assert binding.srbe_sync_status(sysm.h) == 0, binding.srbe_last_error(sysm.h)
        n = sysm.n_ele
        ks = out["kset"].cpu().numpy().reshape(R, -1, 3)
        Qg, bg, Eg = out["Q"].cpu().numpy(), out["b"].cpu().numpy(), out["E"].cpu().numpy()
        for r in SAMPLED:
            ref = oracle_step(p, batch["solver"], int(seeds[r]), step, wb["ion_pos"][r], wb["ion_q"][r],
                              wb["ele_pos"], wb["ele_side"], float(wb["dpsi"][r]))
            assert np.array_equal(ks[r], ref["kset"]), r
            F = forces_from_soa(out["F"], off, r)
            errF = rel_rms(F, ref["F"])
            errb = rel_rms(bg[r * n:(r + 1) * n], ref["b"])
            errQ = rel_rms(Qg[r * n:(r + 1) * n], ref["Q"])
            scale = energy_scale(p, ref["kset"], wb["ion_pos"][r], wb["ion_q"][r], wb["ele_side"],
                                 float(wb["dpsi"][r]), ref["Q"], ref["b"])
            errE = abs(float(Eg[r]) - ref["E"]) / scale
            print(f"replica {r}: F {errF:.2e} b {errb:.2e} Q {errQ:.2e} E {errE:.2e}", flush=True)
            assert errF < 1e-5, r
            assert errb < 3e-5 and errQ < 3e-5, r
            assert errE < 1e-6, r
            assert abs(Qg[r * n:(r + 1) * n].sum()) < 1e-9 * np.abs(Qg[r * n:(r + 1) * n]).sum(), r
    finally:
        gr.close()


def test_fp64_paper_cell(batch):
    from paper_2509_24742_amd import binding
    wb, p, sysm = batch["wb"], batch["p"], batch["sys"]
    r = 17
    off, xyz, q, dp, sd = _inputs(wb, [r], [2100 + r])
    out = sysm.step(off, xyz, q, dp, sd, 5, precision=0)
    torch.cuda.synchronize()
    assert binding.srbe_sync_status(sysm.h) == 0, binding.srbe_last_error(sysm.h)
    ref = oracle_step(p, batch["solver"], 2100 + r, 5, wb["ion_pos"][r], wb["ion_q"][r], wb["ele_pos"],
                      wb["ele_side"], float(wb["dpsi"][r]))
    assert np.array_equal(out["kset"].cpu().numpy().reshape(-1, 3), ref["kset"])
    F = forces_from_soa(out["F"], off, 0)
    eF, eb, eQ = rel_inf(F, ref["F"]), rel_inf(out["b"].cpu().numpy(), ref["b"]), rel_inf(out["Q"].cpu().numpy(),
                                                                                          ref["Q"])
    eE = abs(float(out["E"][0]) - ref["E"]) / abs(ref["E"])
    print(f"fp64 paper cell: F {eF:.2e} b {eb:.2e} Q {eQ:.2e} E {eE:.2e}", flush=True)
    assert eF < 1e-11 and eb < 1e-11 and eE < 1e-11
    assert eQ < 1e-10
