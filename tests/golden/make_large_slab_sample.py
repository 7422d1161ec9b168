"""Writes large_slab_sample.json (P = 500) and large_slab_sample_P2000.json (P = 2000): FP64
oracle values at sampled targets of the full-size large slab.

The inputs are the seeded full-size large slab (``workloads.large_slab()``: 2 x 256 x 256
square walls, 917,504 ions, 30 x 30 x 100 nm, M = 64, P = 500 or 2000), fixed electrode charges
Q_j = side_j 0.004 + 0.001 N(0, 1) (numpy generator seed 9) and the k-set that the
sampler draws for (seed 81, step 3).  The values are b* (Eq. (24) with the exact slab and
real-space parts) at 64 sampled electrodes and the total ion force (Eq. (25) with the slab
and real-space forces) on 64 sampled ions (generator seed 4), from ``oracle.srbe``'s
sampled-target forms.  Run from the repository root:

    python tests/golden/make_large_slab_sample.py [P]

(P = 500 by default; about two minutes on one core, P = 2000 about four).
"""

import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import ewald, sampler, srbe  # noqa: E402
from paper_2509_24742_amd import workloads  # noqa: E402  (inputs only)

SEED, STEP, Q_SEED, SAMPLE_SEED, N_SAMPLE = 81, 3, 9, 4, 64


def golden_name(P):
    return "large_slab_sample.json" if P == 500 else f"large_slab_sample_P{P}.json"


def inputs(P=500):
    w = workloads.large_slab(P=P)
    rng = np.random.default_rng(Q_SEED)
    Q = w["ele_side"] * 0.004 + 0.001 * rng.normal(size=len(w["ele_side"]))
    rs = np.random.default_rng(SAMPLE_SEED)
    ii = np.sort(rs.choice(len(w["ion_q"]), N_SAMPLE, replace=False))
    ie = np.sort(rs.choice(len(w["ele_side"]), N_SAMPLE, replace=False))
    return w, Q, ii, ie


def main(P=500):
    w, Q, ii, ie = inputs(P)
    wp = w["params"]
    p = ewald.Params(Lx=wp["Lx"], Ly=wp["Ly"], H=wp["H"], lam=wp["lam"], alpha=wp["alpha"], eta=wp["eta"],
                     rc=wp["rc"], coulomb_k=wp["coulomb_k"], M=int(wp["M"]), P=int(wp["P"]), kspace_tol=1e-16)
    ks, _ = sampler.draw_kset(p, SEED, 0, STEP)
    b = srbe.srbe_b_at(p, ks, w["ion_pos"], w["ion_q"], w["ele_pos"], ie)
    F = srbe.srbe_ion_forces_at(p, ks, w["ion_pos"], w["ion_q"], w["ele_pos"], Q, ii)
    out = dict(seed=SEED, step=STEP, ion_index=ii.tolist(), ele_index=ie.tolist(), b=b.tolist(), F=F.tolist(),
               n_ion=int(len(w["ion_q"])), n_ele=int(len(w["ele_side"])),
               ion_pos_checksum=float(np.sum(w["ion_pos"] * np.arange(1, 4))))
    out["P"] = int(wp["P"])
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), golden_name(P))
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {path}")


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 500)
