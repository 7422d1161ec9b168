"""Voltage sweep of the paper-shaped cell under positional jitter.

    python -m paper_2509_24742_amd.voltage_sweep [--steps 1000] [--sigma 0.01] [--precision fp32]

The paper-shaped cell (3.4 x 3.7 x 12 nm, three honeycomb layers per electrode, 320
three-site cations + 320 anions; alpha = 3.5/nm, M = 13, P = 200) at the nine potential
differences 0, 0.5, ..., 4 V, one replica each with its own sampler seed, all nine in one
captured step.  Every step the SRBE step runs (fresh sample, constant-potential charges,
forces, energy) and then every site moves by an N(0, sigma^2) displacement per axis (x, y
wrap; z reflects at 1.07 nm and H - 1.07 nm, the placement bounds), so that no phase or
structure factor can be reused from one step to the next.  The jitter is the library's
Langevin update (srbe_langevin_update) with zero force, unit mass, gamma dt / m = 1 (the
velocity is replaced by the kick each step) and beta = 2 / sigma^2 with dt = 1, so a
site moves by the previous step's kick, an N(0, sigma^2) per axis from the update's
Philox stream.  It moves the first replica's sites, and the other replicas take a copy,
so that all nine voltages see the same ions at every step and differ only in dpsi and
in their samples.

Reports, per voltage, the mean and standard deviation over the steps of the charge on the
negative electrode Q_neg, and of Q_neg minus the 0 V replica's (the same ions: only the
voltage and the sampling noise of the two samples differ); the slope of the mean Q_neg
against dpsi (the cell's capacitance at fixed ions); and the time per step of the
nine-replica batch (the SRBE step and the jitter: a graph replay and eager launches).
"""

import argparse
import json
import sys
import time

import numpy as np

VOLTAGES = [0.5 * i for i in range(9)]


def run(steps=1000, sigma=0.01, precision="fp32", seed=1001):
    import torch

    import paper_2509_24742_amd as srbe_amd
    from paper_2509_24742_amd import binding
    from paper_2509_24742_amd import workloads as wl

    w = wl.paper_cell(seed=seed)
    R = len(VOLTAGES)
    wp = dict(w["params"], kspace_tol=1e-16)
    sysm = srbe_amd.System(wp, w["ele_pos"], w["ele_side"])
    dev = torch.device("cuda")
    n1 = len(w["ion_q"])
    N = R * n1
    off = np.arange(R + 1, dtype=np.int64) * n1
    pos = np.tile(w["ion_pos"], (R, 1))
    xyz = torch.tensor(np.ascontiguousarray(pos.T).ravel(), dtype=torch.float64, device=dev)
    q = torch.tensor(np.tile(w["ion_q"], R), dtype=torch.float64, device=dev)
    dpsi = torch.tensor(VOLTAGES, dtype=torch.float64, device=dev)
    seeds = torch.tensor(5000 + np.arange(R), dtype=torch.int64, device=dev).view(torch.uint64)
    vel = torch.zeros(3 * N, dtype=torch.float64, device=dev)
    F0 = torch.zeros(3 * N, dtype=torch.float64, device=dev)  # the jitter's force: none
    mass = torch.ones(N, dtype=torch.float64, device=dev)
    prec = srbe_amd.SRBE_FP32 if precision == "fp32" else srbe_amd.SRBE_FP64
    gr = sysm.capture(off, xyz, q, dpsi, seeds, 0, precision=prec, want_b=False, want_kset=False)
    n = sysm.n_ele
    neg = torch.tensor(np.asarray(w["ele_side"]) < 0, device=dev)
    H = wp["H"]
    qneg = torch.empty((steps, R), dtype=torch.float64, device=dev)

    x3 = xyz.view(3, R, n1)
    x0 = x3[:, 0, :].contiguous()  # the first replica's sites, moved by the jitter
    v0, F00, m0 = vel[:3 * n1], F0[:3 * n1], mass[:n1]

    def one(k):
        o = gr.launch()
        qneg[k] = (o["Q"].view(R, n) * neg).sum(dim=1)
        binding.srbe_langevin_update(x0, v0, F00, m0, 1.0, 2.0 / sigma ** 2, 1.0, wp["Lx"], wp["Ly"], 1.07,
                                     H - 1.07, 4242, k)
        x3.copy_(x0[:, None, :].expand(3, R, n1))

    for k in range(min(10, steps)):  # warm-up (its charges are overwritten below)
        one(k)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.time()
    e0.record()
    for k in range(steps):
        one(k)
    e1.record()
    torch.cuda.synchronize()
    wall = time.time() - t0
    code = srbe_amd.srbe_sync_status(sysm.h)
    if code != 0:
        raise RuntimeError(srbe_amd.srbe_last_error(sysm.h))
    Qn = qneg.cpu().numpy()
    dQ = Qn - Qn[:, :1]
    gr.close()
    sysm.close()
    return {"voltages_V": VOLTAGES, "steps": steps, "sigma_nm": sigma, "precision": precision,
            "Q_neg_mean": [float(x) for x in Qn.mean(axis=0)], "Q_neg_sd": [float(x) for x in Qn.std(axis=0)],
            "Q_neg_minus_0V_mean": [float(x) for x in dQ.mean(axis=0)],
            "Q_neg_minus_0V_sd": [float(x) for x in dQ.std(axis=0)],
            "capacitance_e_per_V": float(-np.polyfit(VOLTAGES, Qn.mean(axis=0), 1)[0]),
            "ms_per_step_9_replicas": e0.elapsed_time(e1) / steps, "wall_s": wall}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--sigma", type=float, default=0.01)
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    args = ap.parse_args()
    print(json.dumps(run(args.steps, args.sigma, args.precision)), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
