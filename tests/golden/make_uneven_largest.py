"""Writes uneven_largest.json: FP64 oracle values at sampled targets of the largest system
of the uneven batch (``workloads.uneven_batch()`` system 26: 162,990 particles, two 36 x 36
square walls of 1,296 atoms each, 20.84 x 20.84 x 31.87 nm, M = 5, P = 404).

Fixed electrode charges Q_j = side_j 0.004 + 0.001 N(0, 1) (numpy generator seed 9), the
k-set the sampler draws for (seed 4126, step 3); b* at 64 sampled electrodes and the total
ion force on 64 sampled ions (generator seed 4), from ``oracle.srbe``'s sampled-target
forms (the dense electrode matrix of this system is not formed).  Run from the
repository root:

    python tests/golden/make_uneven_largest.py
"""

import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import ewald, sampler, srbe  # noqa: E402
from paper_2509_24742_amd import workloads  # noqa: E402  (inputs only)

SYSTEM, SEED, STEP, Q_SEED, SAMPLE_SEED, N_SAMPLE = 26, 4126, 3, 9, 4, 64


def inputs():
    w = workloads.uneven_batch(place={SYSTEM})[SYSTEM]
    rng = np.random.default_rng(Q_SEED)
    Q = w["ele_side"] * 0.004 + 0.001 * rng.normal(size=len(w["ele_side"]))
    rs = np.random.default_rng(SAMPLE_SEED)
    ii = np.sort(rs.choice(len(w["ion_q"]), N_SAMPLE, replace=False))
    ie = np.sort(rs.choice(len(w["ele_side"]), N_SAMPLE, replace=False))
    return w, Q, ii, ie


def main():
    w, Q, ii, ie = inputs()
    wp = w["params"]
    p = ewald.Params(Lx=wp["Lx"], Ly=wp["Ly"], H=wp["H"], lam=wp["lam"], alpha=wp["alpha"], eta=wp["eta"],
                     rc=wp["rc"], coulomb_k=wp["coulomb_k"], M=int(wp["M"]), P=int(wp["P"]), kspace_tol=1e-16)
    ks, _ = sampler.draw_kset(p, SEED, 0, STEP)
    b = srbe.srbe_b_at(p, ks, w["ion_pos"], w["ion_q"], w["ele_pos"], ie)
    F = srbe.srbe_ion_forces_at(p, ks, w["ion_pos"], w["ion_q"], w["ele_pos"], Q, ii)
    out = dict(system=SYSTEM, seed=SEED, step=STEP, ion_index=ii.tolist(), ele_index=ie.tolist(), b=b.tolist(),
               F=F.tolist(), n_ion=int(len(w["ion_q"])), n_ele=int(len(w["ele_side"])),
               ion_pos_checksum=float(np.sum(w["ion_pos"] * np.arange(1, 4))))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "uneven_largest.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {path}")


if __name__ == "__main__":
    main()
