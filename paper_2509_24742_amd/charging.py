"""Charging of the paper-shaped cell after a voltage step, by SRBE-driven Langevin dynamics.

    python -m paper_2509_24742_amd.charging [--replicas 16] [--equil 20000] [--steps 200000]
                                            [--every 10000] [--P 50] [--M 13] [--gamma 1]
                                            [--alpha 1.87] [--rc 1.6] [--precision fp32]

The analogue of the paper's charging curve (Sec. 4, Fig. 2) on the paper-shaped cell
(3.4 x 3.7 x 12 nm, three honeycomb layers per electrode, 320 three-site cations and 320
anions) with the paper's dynamics parameters: alpha = 1.87/nm, rc = 1.6 nm, M = 13,
P = 50, 500 K, dt = 1 fs.  Each replica (its own placement and seeds) is first run at
dpsi = 0 for --equil steps, then dpsi steps to 2 V and the charge on the negative
electrode, Q_neg(t), is averaged over every window of --every steps.  The dynamics are
the Euler-Maruyama Langevin update of Sec. 3 with friction --gamma (eV ps/nm^2; 1 gives
a velocity relaxation time m/gamma of about 1.5 ps for the anion), positions moved with
the updated velocity (the symplectic ordering of the update; as printed, r + v^n dt gains
energy on the stiff contacts, by 1 + (omega dt)^2 per step, and the dynamics run away),
driven by the SRBE forces plus a stand-in short-range force field (the paper's is not
given): WCA between molecules (eps = 0.05 eV, sigma = 0.3 nm), 9-3 walls at the innermost
electrode layers (eps = 0.2 eV, sigma = 0.45 nm) and harmonic bonds (500 eV/nm^2) holding
each cation's three sites, with reflecting bounds 1 nm from the box ends behind the walls.
The random-batch force noise heats the ions in proportion to dt Var(F*) / gamma; with the
paper's alpha it stays far below the thermostat's control (the kinetic temperature is
reported), while with alpha = 3.5/nm at P = 50 the larger Fourier share of the forces
overheats them at small gamma.  Units: nm, ps, e, V, eV; masses in amu enter as
m / 96.485 (so that eV/nm / mass is nm/ps^2).  Every replica runs in one captured
dynamics step (srbe_md_graph_create) replayed once per time step.

Prints, per window, the mean over the replicas of their window-averaged Q_neg and its
standard error over the replicas, the median per-site kinetic temperature (0.79 T for a
Maxwell distribution) and the count of sites above 100 kT.
"""

import argparse
import json
import sys
import time

import numpy as np

AMU_PER_EV_PS2_NM2 = 96.485  # 1 eV / (amu nm^2 / ps^2)
KB_EV = 8.617333262e-5


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--replicas", type=int, default=16)
    ap.add_argument("--equil", type=int, default=20000)
    ap.add_argument("--steps", type=int, default=200000)
    ap.add_argument("--every", type=int, default=10000)
    ap.add_argument("--gamma", type=float, default=1.0)
    ap.add_argument("--dt", type=float, default=0.001, help="time step (ps)")
    ap.add_argument("--wca-eps", type=float, default=0.05, help="WCA energy (eV)")
    ap.add_argument("--printed-order", action="store_true",
                    help="move the positions with the old velocity, as the update is printed (unstable on the "
                         "stiff contacts; the default moves them with the new velocity)")
    ap.add_argument("--P", type=int, default=50)
    ap.add_argument("--M", type=int, default=13, help="deterministic kz modes |m| <= M")
    ap.add_argument("--alpha", type=float, default=1.87, help="Ewald splitting (1/nm)")
    ap.add_argument("--rc", type=float, default=1.6, help="real-space cutoff (nm)")
    ap.add_argument("--dpsi", type=float, default=2.0)
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    args = ap.parse_args()
    import torch

    import paper_2509_24742_amd as srbe_amd
    from paper_2509_24742_amd import binding
    from paper_2509_24742_amd import workloads as wl

    R = args.replicas
    wb = wl.replica_batch(R=R)
    top = wl.paper_cell_topology()
    wp = dict(wb["params"], kspace_tol=1e-16, P=args.P, M=args.M, alpha=args.alpha, rc=args.rc)
    sysm = srbe_amd.System(wp, wb["ele_pos"], wb["ele_side"])
    dev = torch.device("cuda")
    n1 = len(wb["ion_q"][0])
    N = R * n1
    off = np.arange(R + 1, dtype=np.int64) * n1
    xyz = torch.tensor(np.ascontiguousarray(np.concatenate(wb["ion_pos"]).T).ravel(), dtype=torch.float64, device=dev)
    q = torch.tensor(np.concatenate(wb["ion_q"]), dtype=torch.float64, device=dev)
    mol = np.concatenate([top["mol"] + r * n1 for r in range(R)]).astype(np.int32)
    bond = np.concatenate([np.where(top["bond"] >= 0, top["bond"] + r * n1, -1) for r in range(R)]).astype(np.int32)
    r0 = np.tile(top["bond_r0"], R)
    mass = np.tile(top["mass"], R) / AMU_PER_EV_PS2_NM2
    T = 500.0
    rng = np.random.default_rng(5)
    vel = rng.normal(size=(3, N)) * np.sqrt(KB_EV * T / mass)[None, :]  # Maxwell-Boltzmann start
    v = torch.tensor(vel.ravel(), dtype=torch.float64, device=dev)
    dp = torch.zeros(R, dtype=torch.float64, device=dev)
    sd = torch.tensor(2100 + np.arange(R), dtype=torch.int64, device=dev).view(torch.uint64)
    H = wp["H"]
    ff = dict(wca_eps=args.wca_eps, wca_sigma=0.3, wall_eps=0.2, wall_sigma=0.45, wall_zlo=0.67, wall_zhi=H - 0.67,
              bond_k=500.0)
    md = dict(ff=ff, gamma=args.gamma, beta=1.0 / (KB_EV * T), dt=args.dt, zlo=1.0, zhi=H - 1.0, noise_seed=77,
              symplectic=0 if args.printed_order else 1)
    n = sysm.n_ele
    Q = torch.empty(R * n, dtype=torch.float64, device=dev)
    F = torch.empty(3 * N, dtype=torch.float64, device=dev)
    prec = srbe_amd.SRBE_FP32 if args.precision == "fp32" else srbe_amd.SRBE_FP64
    # the graph reads these buffers at every replay: they stay referenced until it is destroyed
    mass_t, mol_t = torch.tensor(mass, device=dev), torch.tensor(mol, device=dev)
    bond_t, r0_t = torch.tensor(bond, device=dev), torch.tensor(r0, device=dev)
    gr = binding.srbe_md_graph_create(sysm.h, prec, off, xyz, v, q, mass_t, mol_t, bond_t, r0_t, dp, sd, 0, md, Q, F)
    neg = torch.tensor(np.asarray(wb["ele_side"]) < 0, device=dev)

    acc = torch.zeros(R, dtype=torch.float64, device=dev)  # Q_neg summed over the current window

    def report(k, dpsi):
        qn = acc.cpu().numpy() / args.every
        acc.zero_()
        ke = (torch.tensor(mass, device=dev)[None, :] * v.view(3, N) ** 2).sum(dim=0).cpu().numpy() / 3.0
        row = {"t_end_ps": round(k * md["dt"], 4), "window_ps": args.every * md["dt"], "dpsi": dpsi,
               "Q_neg_mean": float(qn.mean()), "Q_neg_se": float(qn.std(ddof=1) / np.sqrt(R)),
               "kinetic_T_median_K": float(np.median(ke)) / KB_EV,
               "sites_above_100kT": int(np.sum(ke > 100.0 * KB_EV * T))}
        print(json.dumps(row), flush=True)
        return row

    t0 = time.time()
    for k in range(-args.equil + 1, 1):  # at 0 V; the last window before the voltage step is reported
        binding.srbe_graph_launch(gr)
        acc += (Q.view(R, n) * neg).sum(dim=1)
        if k % args.every == 0 and k > -args.equil + args.every - 1:
            report(k, 0.0)
    dp.fill_(args.dpsi)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for k in range(1, args.steps + 1):
        binding.srbe_graph_launch(gr)
        acc += (Q.view(R, n) * neg).sum(dim=1)
        if k % args.every == 0:
            report(k, args.dpsi)
    e1.record()
    torch.cuda.synchronize()
    code = binding.srbe_sync_status(sysm.h)
    if code != 0:
        raise RuntimeError(binding.srbe_last_error(sysm.h))
    zs = xyz.view(3, N)[2].cpu().numpy()
    vv = v.view(3, N).cpu().numpy()
    kT = float(np.mean(mass[None, :] * vv * vv))  # equipartition: <m v^2> = kT per component
    print(json.dumps({"replicas": R, "P": args.P, "M": int(wp["M"]), "alpha": args.alpha, "rc": args.rc,
                      "precision": args.precision,
                      "gamma": args.gamma, "kinetic_T_K": kT / KB_EV,
                      "ms_per_dynamics_step_all_replicas": e0.elapsed_time(e1) / args.steps,
                      "wall_s": time.time() - t0, "z_range_nm": [float(zs.min()), float(zs.max())]}), flush=True)
    binding.srbe_graph_destroy(gr)
    sysm.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
