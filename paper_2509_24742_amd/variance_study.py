"""Static variance study of the SRBE estimator (Sec. 3, Remark 3.1; Table 1's quantities).

For one fixed configuration, the charge on the negative electrode and the ion forces
of a step are random through the sampled modes only.  One step of R replicas of the
same configuration with R different seeds draws R independent samples at once.  For
each truncation M of the deterministic kz modes and batch size P this reports the mean
and standard deviation over the samples of

  Q_neg  the total charge on the negative electrode (Table 1's quantity), and
  F      the ion forces, as the relative fluctuation
         sqrt(sum_i,d var(F_id) / sum_i,d mean(F_id)^2).

Remark 3.1: the charge variance falls with a Gaussian rate in M until M reaches the
aspect ratio lambda mu, then levels off; it scales as 1/P.

    python -m paper_2509_24742_amd.variance_study [--samples 256] [--workload paper|tiny]
"""

import argparse
import math

import numpy as np

from . import SRBE_FP32, SRBE_FP64, System
from . import workloads as wl


def configuration(name):
    w = wl.paper_cell() if name == "paper" else wl.tiny_slab()
    aspect = 3.0 * w["params"]["H"] / max(w["params"]["Lx"], w["params"]["Ly"])
    return w, aspect


def sample_step(w, M, P, samples, precision=SRBE_FP64, dpsi=2.0, seed0=5000, step=0, kspace_tol=1e-16):
    """Q (samples x n_ele) and F (samples x N_ion x 3) of one step of `samples` replicas of w."""
    import torch
    wp = dict(w["params"], M=int(M), P=int(P), kspace_tol=kspace_tol)
    sysm = System(wp, w["ele_pos"], w["ele_side"])
    try:
        n_ion = len(w["ion_q"])
        dev = torch.device("cuda")
        pos = np.tile(np.asarray(w["ion_pos"], dtype=np.float64), (samples, 1))
        off = np.arange(samples + 1, dtype=np.int64) * n_ion
        xyz = torch.tensor(np.ascontiguousarray(pos.T).ravel(), dtype=torch.float64, device=dev)
        q = torch.tensor(np.tile(np.asarray(w["ion_q"], dtype=np.float64), samples), device=dev)
        dp = torch.full((samples,), float(dpsi), dtype=torch.float64, device=dev)
        seeds = np.arange(seed0, seed0 + samples, dtype=np.uint64)
        sd = torch.tensor(seeds.view(np.int64), device=dev).view(torch.uint64)
        out = sysm.step(off, xyz, q, dp, sd, step, precision=precision, want_kset=False)
        torch.cuda.synchronize()
        Q = out["Q"].cpu().numpy().reshape(samples, -1)
        F = out["F"].cpu().numpy().reshape(3, samples, n_ion).transpose(1, 2, 0)
        return Q, F
    finally:
        sysm.close()


def statistics(w, Q, F):
    neg = np.asarray(w["ele_side"]) < 0
    qn = Q[:, neg].sum(axis=1)
    fm = F.mean(axis=0)
    rel_f = math.sqrt(float(F.var(axis=0).sum()) / float((fm ** 2).sum()))
    return dict(q_neg_mean=float(qn.mean()), q_neg_sd=float(qn.std(ddof=1)), force_rel_sd=rel_f)


def study(name="paper", samples=256, Ms=None, Ps=(20, 50, 100, 200), precision=SRBE_FP64):
    w, aspect = configuration(name)
    lm = int(math.ceil(aspect))
    Ms = Ms or sorted({0, 2, 5, lm, int(w["params"]["M"]), 2 * lm})
    rows = []
    for M in Ms:
        for P in Ps:
            Q, F = sample_step(w, M, P, samples, precision=precision)
            rows.append(dict(M=M, P=P, **statistics(w, Q, F)))
    return dict(workload=name, aspect=aspect, samples=samples, rows=rows)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--samples", type=int, default=256)
    ap.add_argument("--workload", choices=["paper", "tiny"], default="paper")
    ap.add_argument("--fp32", action="store_true")
    a = ap.parse_args()
    res = study(a.workload, a.samples, precision=SRBE_FP32 if a.fp32 else SRBE_FP64)
    print(f"{a.workload} cell, aspect ratio {res['aspect']:.2f}, {res['samples']} samples per (M, P)")
    print("| M | P | Q_neg mean | Q_neg SD | force relative SD |")
    print("|---|---|---|---|---|")
    for r in res["rows"]:
        print(f"| {r['M']} | {r['P']} | {r['q_neg_mean']:.4f} | {r['q_neg_sd']:.4f} | {r['force_rel_sd']:.4f} |")


if __name__ == "__main__":
    main()
