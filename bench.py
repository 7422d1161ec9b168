#!/usr/bin/env python
"""Throughput of the SRBE constant-potential step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]

Headline workload ("replica batch"): 64 paper-shaped electrode / ionic-liquid cells
(3.4 x 3.7 x 12 nm, lambda = 3, 2160 electrode atoms in three honeycomb layers per
side, 320 three-site cations + 320 anions = 1280 ion sites; alpha = 3.5 /nm,
eta = 0.0556 nm, rc = 1.2 nm, M = 13, P = 200), one voltage in [0, 4] V and one seed
per replica, all replicas in one srbe_step call, FP32 k-space and real space with
the FP64 charge solve.  One "step" is one full SRBE step (sampling, structure
factors, b*, charge solve, forces, energy) for all 64 replicas; inputs are resident
in HBM.  The FP64 path on a single cell is timed beside it.

Metric: k-particle pairs per second, pairs/step = sum over replicas of
(N_ion + N_ele) (M + P); steps/s and the 1-fs ns/day equivalent are reported too.
Printed as one JSON line.
"""

import argparse
import hashlib
import json
import os
import resource
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

LANE_OPS_PEAK = 256 * 64 * 2.4e9  # VALU lane-ops per second: 256 CUs x 64 lanes x 2.4 GHz
FP64_PEAK = 78.6e12                # FP64 MFMA FLOP/s

# Algorithmic VALU slots per unit of work of each FP32 kernel (a transcendental --
# sin, cos, exp, rsqrt, rcp -- issues at quarter rate and counts 4 slots; sin/cos
# at half rate, 2).  k-space passes, per (particle, mode) pair: exact integer phase
# (3 multiplies + 1 three-way add), int->float + scale (2), sin and cos (4), then
# the accumulation: structure factor 2 FMA; electrode potential 2 FMA; force
# 2 (Im part) + 3 FMA.  Real-space passes, per pair closer than rc: fixed-point
# difference (3 sub, 3 convert, 3 scale), r^2 (3), rsqrt (4), r and alpha r (2),
# t = 1/(1 + x/2) (1 + 4), the degree-9 polynomial (9), exp(-x^2) (2 + 4), erfc/r (3),
# then ion-ion: the force factor (3), potential (1), force (1 + 3) = 49; ion-
# electrode force: 48 (no potential); electrode potential: r^2 from the
# difference (9 + 3), rsqrt, r, x, t, polynomial, exp, erfc/r (30) and 1 FMA = 43.
SLOTS = {"sf_ions": 12, "sf_ele": 12, "ele_potential": 12, "ion_force": 15,
         "real_ii": 49, "real_ie": 48, "real_ele": 43}

# Algorithmic HBM bytes per unit of the memory-bound phases (the step roofline's bytes
# term): records + cell sort per particle (SoA position 24 B and charge 8 B read; 16-byte
# record, key, permutation entry, cell and 16-byte sorted record written); the charge
# copy-out per electrode and replica (Q read, Q, FP32 Q and its cell-sorted copy
# written); the last launch per ion (F, the two real-space sums and the charge read, F
# written).
BYTES = {"cellsort": 24 + 8 + 16 + 4 + 4 + 4 + 16, "post_charges": 8 + 8 + 4 + 4, "energy": 24 + 24 + 24 + 8 + 24}
HBM_PEAK = 8.0e12  # bytes/s
PROF_REPS = 10     # launches of each phase between its timing events

# HBM traffic per launch of the step's kernels, from rocprofv3 FETCH_SIZE and WRITE_SIZE
# runs scaled by the same counters' reading for a plain copy of COPY_BYTES (see the
# profile named below).  The figures hold only for the kernel source they were taken
# on: its SHA-256 is recorded beside them, and a changed source reports null.
COPY_BYTES = 1 << 29
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "kernel_traffic_replica_batch64.md")
# VALU instruction counts per launch (rocprofv3 SQ counters), same SHA-256 rule
COUNTER_PROFILE = os.path.join(ROOT, "profiles", "kernel_counters_replica_batch64.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2509_24742_amd", "csrc", "step_kernels.hip")
# launch parameters chosen by srbe_tune's timing of these workloads on an MI355X
TUNING_CACHE = os.path.join(ROOT, "paper_2509_24742_amd", "tuning_cache.json")


def measured_traffic():
    """{phase: HBM bytes per launch} if the recorded figures match the current kernel source, else {}."""
    try:
        lines = open(TRAFFIC_PROFILE).read().splitlines()
    except OSError:
        return {}
    rec = {}
    for ln in lines:
        if ln.startswith("traffic ") or ln.startswith("source_sha256 "):
            parts = ln.split()
            rec[parts[1] if parts[0] == "traffic" else "sha"] = parts[-1]
    sha = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    if rec.get("sha") != sha:
        return {}
    return {k: float(v) for k, v in rec.items() if k != "sha"}


def measured_counters():
    """{phase: (VALU instructions, ratio to algorithmic, issue fraction)} if recorded for the current source."""
    try:
        lines = open(COUNTER_PROFILE).read().splitlines()
    except OSError:
        return {}
    rec, sha = {}, None
    for ln in lines:
        parts = ln.split()
        if ln.startswith("source_sha256 "):
            sha = parts[-1]
        elif ln.startswith("valu ") and len(parts) == 7:
            rec[parts[1]] = (float(parts[2]), float(parts[4]), float(parts[6]))
    if sha != hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest():
        return {}
    return rec


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--replicas", type=int, default=64)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline and error check")
    ap.add_argument("--no-tune", action="store_true",
                    help="time with the default launch parameters")
    ap.add_argument("--large-slab", type=int, nargs="*", default=[500, 2000], metavar="P",
                    help="batch sizes P at which to time the full-size large slab (917,504 ions, 131,072 electrodes, "
                         "M=64, charges by the lattice solve); reported as large_slab (default: 500 2000)")
    ap.add_argument("--no-large-slab", action="store_true", help="skip the large slab")
    ap.add_argument("--no-uneven", action="store_true",
                    help="skip the uneven batch (32 systems of 2e3-2e5 particles, each its own box, charges by the "
                         "lattice solve), otherwise timed and reported as uneven_batch")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the voltage sweep (the paper-shaped cell at 0..4 V, 1000 steps with 0.01 nm "
                         "positional jitter), otherwise reported as voltage_sweep")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="first run a plain device copy of COPY_BYTES (the reference that HBM byte counters "
                         "are scaled by)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the library has no multi-GPU "
              f"path (replicas would shard across GPUs without communication)", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2509_24742_amd as srbe_amd
    from paper_2509_24742_amd import workloads as wl

    dev = torch.device("cuda:0")
    if args.traffic_probe:
        src = torch.empty(COPY_BYTES // 8, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    R = args.replicas
    t0 = time.time()
    wb = wl.replica_batch(R=R)
    gen_s = time.time() - t0
    log(f"generated {R} replicas in {gen_s:.1f} s")
    wp = dict(wb["params"], kspace_tol=1e-16)
    t0 = time.time()
    sysm = srbe_amd.System(wp, wb["ele_pos"], wb["ele_side"])
    setup_s = time.time() - t0
    log(f"electrode set-up (A, Cholesky, J A^-1) in {setup_s:.2f} s")
    n_ele = sysm.n_ele
    sizes = [len(q) for q in wb["ion_q"]]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    pos = np.concatenate(wb["ion_pos"])
    xyz = torch.tensor(np.ascontiguousarray(pos.T).ravel(), dtype=torch.float64, device=dev)
    q = torch.tensor(np.concatenate(wb["ion_q"]), dtype=torch.float64, device=dev)
    dpsi = torch.tensor(wb["dpsi"], dtype=torch.float64, device=dev)
    seeds = torch.tensor(2100 + np.arange(R), dtype=torch.int64, device=dev).view(torch.uint64)
    M, P = int(wp["M"]), int(wp["P"])
    K = M + P
    pairs_per_step = int(sum(n + n_ele for n in sizes)) * K
    paper_pairs_per_step = int(sum(n + n_ele for n in sizes)) * (2 * M + P)

    out = None
    stream = torch.cuda.current_stream()
    log("counting real-space pairs ...")
    npair_ii, npair_ie = count_pairs(wb, wp)

    def run(steps, first, prec, offs, x, qq, dp, sd, o):
        for i in range(steps):
            o = sysm.step(offs, x, qq, dp, sd, first + i, precision=prec, want_kset=False, out=o)
        return o

    def timed(prec, offs, x, qq, dp, sd):
        o = run(args.warmup, 0, prec, offs, x, qq, dp, sd, None)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        o = run(args.steps, args.warmup, prec, offs, x, qq, dp, sd, o)
        e1.record(stream)
        torch.cuda.synchronize()
        code = srbe_amd.srbe_sync_status(sysm.h)
        if code != 0:
            raise RuntimeError(srbe_amd.srbe_last_error(sysm.h))
        return e0.elapsed_time(e1) / args.steps, o

    def timed_graph(prec, offs, x, qq, dp, sd):
        gr = sysm.capture(offs, x, qq, dp, sd, 0, precision=prec, want_kset=False)
        for _ in range(args.warmup):
            gr.launch()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            gr.launch()
        e1.record(stream)
        torch.cuda.synchronize()
        code = srbe_amd.srbe_sync_status(sysm.h)
        if code != 0:
            raise RuntimeError(srbe_amd.srbe_last_error(sysm.h))
        gr.close()
        return e0.elapsed_time(e1) / args.steps

    # single-cell inputs (replica 0)
    off1 = np.array([0, sizes[0]], dtype=np.int64)
    xyz1 = torch.tensor(np.ascontiguousarray(wb["ion_pos"][0].T).ravel(), dtype=torch.float64, device=dev)
    q1 = torch.tensor(wb["ion_q"][0], dtype=torch.float64, device=dev)
    dpsi1, seeds1 = dpsi[:1].contiguous(), seeds[:1].contiguous()

    # ---- launch-parameter tuning (srbe_tune), outside the timed region
    tuning = None
    if not args.no_tune:
        t0 = time.time()
        tuning = {"source": "shipped choices (tuning_cache.json)"}
        for name, prec, offs, x, qq, dp, sd in [("fp32_batch", srbe_amd.SRBE_FP32, off, xyz, q, dpsi, seeds),
                                                ("fp64_single_cell", srbe_amd.SRBE_FP64, off1, xyz1, q1, dpsi1, seeds1),
                                                ("fp32_single_cell", srbe_amd.SRBE_FP32, off1, xyz1, q1, dpsi1, seeds1)]:
            t = sysm.tune(offs, x, qq, dp, sd, precision=prec, cache=TUNING_CACHE, tune_missing=False)
            tuning[name] = {"params": dict(zip(srbe_amd.SRBE_TUNE_NAMES, t["params"])),
                            "ms_default": t["ms_default"], "ms_tuned": t["ms_tuned"], "from_cache": t["cached"]}
        tuning["seconds"] = time.time() - t0
        log(f"launch parameters ({tuning['source']}) in {tuning['seconds']:.2f} s: {tuning['fp32_batch']['params']}")

    # ---- headline: FP32, all replicas in one step, replayed as a captured graph
    ms_fp32 = timed_graph(srbe_amd.SRBE_FP32, off, xyz, q, dpsi, seeds)
    log(f"FP32 batch (graph): {ms_fp32 * 1e3:.1f} us/step")
    ms_fp32_eager, out = timed(srbe_amd.SRBE_FP32, off, xyz, q, dpsi, seeds)
    log(f"FP32 batch (eager): {ms_fp32_eager * 1e3:.1f} us/step")
    ms_bf16 = timed_graph(srbe_amd.SRBE_BF16, off, xyz, q, dpsi, seeds)
    log(f"BF16 hi/lo structure-factor variant (graph): {ms_bf16 * 1e3:.1f} us/step")

    # ---- per-phase durations (HIP events recorded by the library on the stream that runs
    # each phase; every phase but the last is launched PROF_REPS times between its events,
    # so the events' own cost is spread over the launches: the figures are per launch)
    srbe_amd.srbe_profile_enable(sysm.h, PROF_REPS)
    nprof = min(args.steps, 20)
    run(nprof, args.warmup + args.steps, srbe_amd.SRBE_FP32, off, xyz, q, dpsi, seeds, out)
    torch.cuda.synchronize()
    prof = srbe_amd.srbe_profile_read(sysm.h)
    srbe_amd.srbe_profile_enable(sysm.h, False)
    phases = {k: {"avg_us": 1e3 * v[0] / v[1], "launches": v[1]} for k, v in prof.items() if v[1]}

    # ---- FP64 plain path on one cell
    ms_fp64_1 = timed_graph(srbe_amd.SRBE_FP64, off1, xyz1, q1, dpsi1, seeds1)
    pairs_1 = (sizes[0] + n_ele) * K
    # FP32 on a single cell, for the batching gain
    ms_fp32_1 = timed_graph(srbe_amd.SRBE_FP32, off1, xyz1, q1, dpsi1, seeds1)
    log(f"single cell: FP64 {ms_fp64_1 * 1e3:.1f} us/step, FP32 {ms_fp32_1 * 1e3:.1f} us/step")

    # ---- roofline of the dominant kernel (longest phase with a roofline figure)
    # ion-ion pairs are counted unordered (Eq. (13) sums each pair once), although the
    # pass evaluates every pair from both ions
    npair_ii_u = npair_ii // 2
    units = {
        "sf_ions": sum(sizes) * K,
        "sf_ele": R * n_ele * K,
        "ele_potential": R * n_ele * K,
        "ion_force": sum(sizes) * K,
        "real_ii": npair_ii_u,
        "real_ie": npair_ie,
        "real_ele": npair_ie,
    }
    gemm_flop = 2.0 * (n_ele + 1) * n_ele * R
    gemm_bytes = 8.0 * (n_ele + 1) * ((n_ele + 31) // 32 * 32)  # S_ext, read once
    cands = [k for k in list(SLOTS) + ["cp_gemm"] if k in phases]
    kdom = max(cands, key=lambda k: phases[k]["avg_us"])
    dur = phases[kdom]["avg_us"] * 1e-6
    if kdom == "cp_gemm":
        ach = gemm_flop / dur
        roofline = {"bound": "mfma", "kernel": kdom, "achieved": ach / 1e12, "peak": FP64_PEAK / 1e12,
                    "unit": "TFLOP/s", "frac": ach / FP64_PEAK, "traffic": None}
    else:
        ach = units[kdom] * SLOTS[kdom] / dur
        roofline = {"bound": "alu", "kernel": kdom, "achieved": ach / 1e12, "peak": LANE_OPS_PEAK / 1e12,
                    "unit": "TVALUop/s", "frac": ach / LANE_OPS_PEAK, "traffic": None,
                    "work": f"{units[kdom]} {'unordered ion-ion pairs' if kdom == 'real_ii' else 'units'} x "
                            f"{SLOTS[kdom]} VALU slots per launch",
                    "us_per_launch": round(dur * 1e6, 2)}
    traffic = measured_traffic()
    if kdom in traffic:
        roofline["traffic"] = traffic[kdom]
        roofline["traffic_unit"] = "HBM bytes per launch"
    counters = measured_counters()
    if kdom in counters:
        vi, ratio, issue = counters[kdom]
        roofline["valu_instructions_per_launch"] = vi
        roofline["valu_instructions_over_algorithmic"] = ratio
        roofline["valu_issue_fraction"] = issue
    if kdom.startswith("real"):
        tb = f"{traffic[kdom] / dur / 1e12:.2f} TB/s" if kdom in traffic else "unmeasured"
        ev = (f"ALU-issue bound, not HBM: HBM traffic per launch {tb} of 8 TB/s "
              f"(profiles/kernel_traffic_replica_batch64.md)")
        if kdom in counters:
            ev += (f"; {counters[kdom][0]:.3g} VALU wave instructions per launch, {counters[kdom][1]:.1f}x the "
                   f"algorithmic count, issued at {counters[kdom][2]:.2f} of one per CU per cycle "
                   f"(profiles/kernel_counters_replica_batch64.md): the candidate tests and bookkeeping, "
                   f"not the pair terms, take the issue slots")
        roofline["bound_evidence"] = ev
    other = {}
    for k in cands:
        d = phases[k]["avg_us"] * 1e-6
        if k == "cp_gemm":
            other[k] = {"us": round(d * 1e6, 2), "frac": round(gemm_flop / d / FP64_PEAK, 4), "of": "FP64 MFMA peak"}
        else:
            other[k] = {"us": round(d * 1e6, 2), "frac": round(units[k] * SLOTS[k] / d / LANE_OPS_PEAK, 4),
                        "of": "VALU slot peak"}
    top = max(phases, key=lambda k: phases[k]["avg_us"])
    # step roofline: every phase at its own bound, one after another
    ideal = {k: units[k] * SLOTS[k] / LANE_OPS_PEAK for k in SLOTS}
    ideal["cp_gemm"] = max(gemm_flop / FP64_PEAK, gemm_bytes / HBM_PEAK)
    ideal["cellsort"] = sum(sizes) * BYTES["cellsort"] / HBM_PEAK
    ideal["post_charges"] = R * n_ele * BYTES["post_charges"] / HBM_PEAK
    ideal["energy"] = sum(sizes) * BYTES["energy"] / HBM_PEAK
    ideal_us = {k: round(v * 1e6, 3) for k, v in ideal.items()}
    step_roof = {"ideal_us_per_step": round(sum(ideal.values()) * 1e6, 2), "ideal_us_by_phase": ideal_us,
                 "step_frac": sum(ideal.values()) / (ms_fp32 * 1e-3),
                 "definition": "sum over the step's phases of max(algorithmic bytes / 8 TB/s, algorithmic VALU "
                               "slots / 39.3 T lane-ops/s, FP64 MFMA flops / 78.6 TFLOP/s), divided by ms_per_step "
                               "(the sampler is left out: under 0.1 us of work)"}

    result = {
        "metric": "SRBE k-particle pairs/s (FP32-batched step; FP64 plain beside it)",
        "value": pairs_per_step / (ms_fp32 * 1e-3),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_fp32,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (k-space, real space); f64 (charge solve, energy)",
        "data": "synthetic",
        "config": {"workload": f"replica batch: {R} paper-shaped cells (1280 ion sites + 2160 electrode atoms), "
                               f"M={M}, P={P}, alpha=3.5/nm, rc=1.2 nm", "replicas": R,
                   "pairs_per_step": pairs_per_step, "paper_pair_count_per_step": paper_pairs_per_step},
        "steps_per_s": 1e3 / ms_fp32,
        "ns_per_day_equiv_1fs": 1e3 / ms_fp32 * 0.0864,
        "fp64_plain_single_cell": {"ms_per_step": ms_fp64_1, "pairs_per_s": pairs_1 / (ms_fp64_1 * 1e-3),
                                   "steps_per_s": 1e3 / ms_fp64_1},
        "fp32_single_cell": {"ms_per_step": ms_fp32_1, "pairs_per_s": pairs_1 / (ms_fp32_1 * 1e-3)},
        "speedup_vs_fp64_plain_pairs_per_s": (pairs_per_step / ms_fp32) / (pairs_1 / ms_fp64_1),
        "roofline": roofline,
        "kernel_rooflines": other,
        "ms_per_step_eager": ms_fp32_eager,
        "step_roofline": step_roof,
        "real_space_pairs_per_step": {"ion_ion_unordered": npair_ii_u, "ion_electrode": npair_ie},
        "phases_us_per_launch": {k: round(v["avg_us"], 2) for k, v in phases.items()},
        "slowest_phase": top,
        "setup_s": setup_s,
        "workload_generation_s": gen_s,
        "launch_tuning": tuning,
    }

    if args.large_slab and not args.no_large_slab:
        result["large_slab"] = large_slab_bench(args, srbe_amd, stream)
    if not args.no_uneven:
        result["uneven_batch"] = uneven_bench(args, srbe_amd, stream)
    if not args.no_sweep:
        # the paper-shaped cell at 0, 0.5, ..., 4 V for 1000 steps with 0.01 nm jitter per step
        from paper_2509_24742_amd import voltage_sweep
        log("voltage sweep (9 voltages x 1000 jittered steps) ...")
        result["voltage_sweep"] = voltage_sweep.run(steps=1000, sigma=0.01, precision="fp32")

    if not args.no_cpu:
        o = sysm.step(off, xyz, q, dpsi, seeds, 0, precision=srbe_amd.SRBE_FP32, want_kset=False)
        torch.cuda.synchronize()
        acc = {"off": off, "F": o["F"].cpu().numpy(), "Q": o["Q"].cpu().numpy(), "E": o["E"].cpu().numpy(),
               "b": o["b"].cpu().numpy()}
        side, refs = cpu_side(wb, wp, acc, R, sizes, n_ele, K)
        result.update(side)
        # the BF16 hi/lo structure-factor variant on the same step: an error report
        ob = sysm.step(off, xyz, q, dpsi, seeds, 0, precision=srbe_amd.SRBE_BF16, want_kset=False)
        torch.cuda.synchronize()
        accb = {"off": off, "F": ob["F"].cpu().numpy(), "Q": ob["Q"].cpu().numpy(), "E": ob["E"].cpu().numpy(),
                "b": ob["b"].cpu().numpy()}
        result["bf16_error_vs_fp64_oracle"] = dict(errors_vs_oracle(refs, accb, n_ele),
                                                   ms_per_step=ms_bf16, variant=BF16_VARIANT)
        result["fp32_error_vs_fp64_oracle"].update(error_split(srbe_amd, sysm, wb, wp, refs, off, xyz, q, dpsi,
                                                               seeds, n_ele))
    print(json.dumps(result), flush=True)
    sysm.close()


GOLDEN = os.path.join(ROOT, "tests", "golden")
BF16_VARIANT = ("SRBE_BF16: the FP32 step with each product q cos, q sin of the structure factors formed from "
                "BF16 hi/lo halves (q_hi c_hi + q_hi c_lo + q_lo c_hi, FP32 accumulation), as BF16 matrix cores "
                "would; replicas at their own constant-potential charges, step 0")


def _rel_rms(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def large_slab_bench(args, srbe_amd, stream):
    """Steps of the full-size large slab (one system; the charge update by the lattice solve,
    since the dense one would need a 131,072^2 matrix), FP32 and FP64, as graph replays, at
    each batch size P; the FP32 errors against the FP64 oracle: forces and b* at sampled
    targets of the full size at fixed charges, and charges, energy, forces and b* of the
    constant-potential step of the same recipe at 1/8 scale (values written by the
    scripts in tests/golden)."""
    import json
    import torch
    from paper_2509_24742_amd import workloads as wl
    t0 = time.time()
    w = wl.large_slab()
    gen_s = time.time() - t0
    dev = torch.device("cuda")
    n_ion, n_ele = len(w["ion_q"]), len(w["ele_side"])
    off = np.array([0, n_ion], dtype=np.int64)
    xyz = torch.tensor(np.ascontiguousarray(w["ion_pos"].T).ravel(), dtype=torch.float64, device=dev)
    q = torch.tensor(w["ion_q"], dtype=torch.float64, device=dev)
    dp = torch.tensor([w["dpsi"]], dtype=torch.float64, device=dev)
    steps = max(5, min(args.steps, 50))
    out = {"workload": f"large slab: {n_ion} ions, {n_ele} electrode atoms (2x256x256), 30x30x100 nm, M=64, "
                       f"constant potential (lattice charge solve)", "steps": steps, "workload_generation_s": gen_s}
    rs = np.random.default_rng(9)
    Qfix = w["ele_side"] * 0.004 + 0.001 * rs.normal(size=n_ele)  # the goldens' fixed charges (seed 9)
    for P in args.large_slab:
        wp = dict(w["params"], kspace_tol=1e-16, P=int(P))
        t0 = time.time()
        sysm = srbe_amd.System(wp, w["ele_pos"], w["ele_side"], flags=srbe_amd.SRBE_FLAG_LATTICE_SOLVE)
        res = {"setup_s": time.time() - t0}
        sd = torch.tensor([81], dtype=torch.int64, device=dev).view(torch.uint64)
        pairs = (n_ion + n_ele) * (wp["M"] + wp["P"])
        for name, prec in [("fp32", srbe_amd.SRBE_FP32), ("fp64", srbe_amd.SRBE_FP64)]:
            gr = sysm.capture(off, xyz, q, dp, sd, 0, precision=prec, want_kset=False)
            for _ in range(3):
                gr.launch()
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(steps):
                gr.launch()
            e1.record(stream)
            torch.cuda.synchronize()
            code = srbe_amd.srbe_sync_status(sysm.h)
            if code != 0:
                raise RuntimeError(srbe_amd.srbe_last_error(sysm.h))
            gr.close()
            ms = e0.elapsed_time(e1) / steps
            res[name] = {"ms_per_step": ms, "pairs_per_s": pairs / (ms * 1e-3), "steps_per_s": 1e3 / ms}
            log(f"large slab P={P} {name}: {ms:.3f} ms/step")
        sysm.close()
        res["pairs_per_step"] = pairs
        # FP32 error at the full size: fixed charges, sampled targets
        gname = "large_slab_sample.json" if P == 500 else f"large_slab_sample_P{P}.json"
        gpath = os.path.join(GOLDEN, gname)
        if os.path.exists(gpath):
            with open(gpath) as f:
                ref = json.load(f)
            fixed = srbe_amd.System(wp, w["ele_pos"], w["ele_side"], flags=srbe_amd.SRBE_FLAG_NO_CP)
            sdg = torch.tensor([ref["seed"]], dtype=torch.int64, device=dev).view(torch.uint64)
            o = fixed.step(off, xyz, q, dp, sdg, ref["step"], precision=srbe_amd.SRBE_FP32,
                           Q_in=torch.tensor(Qfix, dtype=torch.float64, device=dev), want_kset=False)
            torch.cuda.synchronize()
            ii, ie = np.asarray(ref["ion_index"]), np.asarray(ref["ele_index"])
            F = o["F"].cpu().numpy().reshape(3, n_ion)[:, ii].T
            b = o["b"].cpu().numpy()[ie]
            res["fp32_error_vs_fp64_oracle_full_size"] = {
                "force_rel_rms": _rel_rms(F, ref["F"]), "b_rel_rms": _rel_rms(b, ref["b"]),
                "targets": f"{len(ii)} ions, {len(ie)} electrodes (fixed charges; {gname})"}
            fixed.close()
        out[f"P{P}"] = res
    # FP32 errors at 1/8 scale, constant potential, every quantity
    mpath = os.path.join(GOLDEN, "large_slab_mid.json")
    if os.path.exists(mpath):
        with open(mpath) as f:
            mref = json.load(f)
        sz = mref["size"]
        for P in args.large_slab:
            if str(P) not in mref:
                continue
            wm = wl.large_slab(P=int(P), **sz)
            wpm = dict(wm["params"], kspace_tol=1e-16)
            sm = srbe_amd.System(wpm, wm["ele_pos"], wm["ele_side"], flags=srbe_amd.SRBE_FLAG_LATTICE_SOLVE)
            nm = len(wm["ion_q"])
            offm = np.array([0, nm], dtype=np.int64)
            xm = torch.tensor(np.ascontiguousarray(wm["ion_pos"].T).ravel(), dtype=torch.float64, device=dev)
            qm = torch.tensor(wm["ion_q"], dtype=torch.float64, device=dev)
            sdm = torch.tensor([mref["seed"]], dtype=torch.int64, device=dev).view(torch.uint64)
            o = sm.step(offm, xm, qm, dp, sdm, mref["step"], precision=srbe_amd.SRBE_FP32, want_kset=False)
            torch.cuda.synchronize()
            r = mref[str(P)]
            ii, ie = np.asarray(mref["ion_index"]), np.asarray(mref["ele_index"])
            Q = o["Q"].cpu().numpy()
            out[f"P{P}"]["fp32_error_vs_fp64_oracle_eighth_scale"] = {
                "charge_rel_rms": _rel_rms(Q, r["Q"]), "energy_rel": abs(float(o["E"][0]) - r["E"]) / abs(r["E"]),
                "force_rel_rms": _rel_rms(o["F"].cpu().numpy().reshape(3, nm)[:, ii].T, r["F"]),
                "b_rel_rms": _rel_rms(o["b"].cpu().numpy()[ie], r["b"]),
                "psibar_abs": abs(float(o["psibar"][0]) - r["psibar"]),
                "system": f"{nm} ions, {len(wm['ele_side'])} electrode atoms (2x32x32), 3.75x3.75x12.5 nm, "
                          f"constant potential; oracle's dense solve (large_slab_mid.json)"}
            sm.close()
    return out


def uneven_bench(args, srbe_amd, stream):
    """One step of each of the 32 uneven-batch systems (each its own box and handle, the
    lattice charge solve), FP32 and FP64: all systems in one batch step with one launch per
    phase (srbe_batch, captured), and beside it the systems' own captured steps spread over
    streams.  FP32 errors against the FP64 oracle: the three smallest systems in full (the
    oracle's dense solve, computed here), the largest at sampled targets (fixed charges;
    tests/golden/uneven_largest.json)."""
    import json
    import torch
    from paper_2509_24742_amd import binding
    from paper_2509_24742_amd import workloads as wl
    t0 = time.time()
    systems = wl.uneven_batch()
    gen_s = time.time() - t0
    dev = torch.device("cuda")
    t0 = time.time()
    items = []
    for k, w in enumerate(systems):
        wp = dict(w["params"], kspace_tol=1e-16)
        sysm = srbe_amd.System(wp, w["ele_pos"], w["ele_side"], flags=srbe_amd.SRBE_FLAG_LATTICE_SOLVE)
        n_ion = len(w["ion_q"])
        items.append(dict(sys=sysm, off=np.array([0, n_ion], dtype=np.int64),
                          xyz=torch.tensor(np.ascontiguousarray(w["ion_pos"].T).ravel(), dtype=torch.float64,
                                           device=dev),
                          q=torch.tensor(w["ion_q"], dtype=torch.float64, device=dev),
                          dp=torch.tensor([w["dpsi"]], dtype=torch.float64, device=dev),
                          sd=torch.tensor([4100 + k], dtype=torch.int64, device=dev).view(torch.uint64),
                          pairs=w["n_total"] * (wp["M"] + wp["P"])))
    setup_s = time.time() - t0
    pairs = sum(it["pairs"] for it in items)
    steps = max(3, min(args.steps, 20))
    out = {"workload": f"uneven batch: {len(items)} systems, {sum(w['n_total'] for w in systems)} particles in all "
                       f"(2e3-2e5 each, log-uniform), aspect 3-12, P = round(100 sqrt(N/1e4)), M = ceil(aspect), "
                       f"constant potential (lattice charge solve)", "systems": len(items), "steps": steps,
           "pairs_per_batch_step": pairs, "workload_generation_s": gen_s, "setup_s": setup_s}
    # the whole batch as one input set (CSR over the systems, one replica each)
    sizes = [len(w["ion_q"]) for w in systems]
    boff = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    sor = np.arange(len(systems), dtype=np.int32)
    bxyz = torch.tensor(np.ascontiguousarray(np.concatenate([w["ion_pos"] for w in systems]).T).ravel(),
                        dtype=torch.float64, device=dev)
    bq = torch.tensor(np.concatenate([w["ion_q"] for w in systems]), dtype=torch.float64, device=dev)
    bdp = torch.tensor([w["dpsi"] for w in systems], dtype=torch.float64, device=dev)
    bsd = torch.tensor(4100 + np.arange(len(systems)), dtype=torch.int64, device=dev).view(torch.uint64)
    n_eles = [len(w["ele_side"]) for w in systems]
    nq, N = int(sum(n_eles)), int(boff[-1])
    bt = binding.srbe_batch_create([it["sys"].h for it in items])

    def timed_replays(launch):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            launch()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    # the systems' own graphs go to S streams (default priority), largest first, each to
    # the stream with the least work so far; the batch step ends when every stream has
    order = sorted(range(len(items)), key=lambda k: -items[k]["pairs"])
    bout = None
    for name, prec in [("fp32", srbe_amd.SRBE_FP32), ("fp64", srbe_amd.SRBE_FP64)]:
        o = dict(Q=torch.empty(nq, dtype=torch.float64, device=dev),
                 F=torch.empty(3 * N, dtype=torch.float64, device=dev),
                 psibar=torch.empty(len(systems), dtype=torch.float64, device=dev),
                 E=torch.empty(len(systems), dtype=torch.float64, device=dev))
        bg = binding.srbe_batch_graph_create(bt, prec, boff, sor, bxyz, bq, bdp, bsd, 0, o["Q"], o["F"], o["psibar"],
                                             energy_out=o["E"])
        for _ in range(2):
            binding.srbe_batch_graph_launch(bg)
        torch.cuda.synchronize()
        ms_batch = timed_replays(lambda: binding.srbe_batch_graph_launch(bg))
        if binding.srbe_batch_sync_status(bt) != 0:
            raise RuntimeError(binding.srbe_batch_last_error(bt))
        binding.srbe_batch_graph_destroy(bg)
        log(f"uneven batch {name}: {ms_batch:.3f} ms per step of all systems (one launch per phase)")
        graphs = [it["sys"].capture(it["off"], it["xyz"], it["q"], it["dp"], it["sd"], 0, precision=prec,
                                    want_kset=False) for it in items]
        for gr in graphs:
            gr.launch()
        torch.cuda.synchronize()
        res = {}
        for S in (1, 4):
            side = [torch.cuda.Stream() for _ in range(S)]
            load, plan = [0] * S, []
            for k in order:
                j = min(range(S), key=lambda u: load[u])
                load[j] += items[k]["pairs"]
                plan.append((k, j))

            def launch_all():
                for k, j in plan:
                    graphs[k].launch(side[j])

            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for st in side:
                st.wait_event(e0)
            for _ in range(steps):
                launch_all()
            for st in side:
                stream.wait_stream(st)
            e1.record(stream)
            torch.cuda.synchronize()
            res[S] = e0.elapsed_time(e1) / steps
        for it in items:
            code = srbe_amd.srbe_sync_status(it["sys"].h)
            if code != 0:
                raise RuntimeError(srbe_amd.srbe_last_error(it["sys"].h))
        for gr in graphs:
            gr.close()
        out[name] = {"ms_per_batch_step": ms_batch, "pairs_per_s": pairs / (ms_batch * 1e-3),
                     "schedule": "one batch step: one launch per phase for all 32 systems (captured)",
                     "per_system_graphs_ms_by_streams": {str(k): round(v, 4) for k, v in res.items()}}
        log(f"uneven batch {name}: per-system graphs over streams {res}")
        if name == "fp32":
            # the replays above ran steps 0, 1, ...: the error check takes an eager batch step at
            # step 0, the oracle's sample
            binding.srbe_batch_step(bt, prec, boff, sor, bxyz, bq, bdp, bsd, 0, o["Q"], o["F"], o["psibar"],
                                    energy_out=o["E"])
            torch.cuda.synchronize()
            if binding.srbe_batch_sync_status(bt) != 0:
                raise RuntimeError(binding.srbe_batch_last_error(bt))
            bout = {k: v.cpu().numpy() for k, v in o.items()}
    binding.srbe_batch_destroy(bt)
    # FP32 errors: the three smallest systems in full against the oracle's dense solve
    from oracle import cp, ewald, sampler, srbe
    errs = {}
    qoff = np.concatenate([[0], np.cumsum(n_eles)])
    F32 = bout["F"].reshape(3, N)
    for k in sorted(range(len(systems)), key=lambda u: systems[u]["n_total"])[:3]:
        w = systems[k]
        wp = w["params"]
        p = ewald.Params(Lx=wp["Lx"], Ly=wp["Ly"], H=wp["H"], lam=wp["lam"], alpha=wp["alpha"], eta=wp["eta"],
                         rc=wp["rc"], coulomb_k=wp["coulomb_k"], M=int(wp["M"]), P=int(wp["P"]), kspace_tol=1e-16)
        ks, _ = sampler.draw_kset(p, 4100 + k, 0, 0)
        ref = srbe.srbe_step(p, cp.Solver(ewald.electrode_matrix(p, w["ele_pos"])), ks, w["ion_pos"], w["ion_q"],
                             w["ele_pos"], w["ele_side"], w["dpsi"])
        errs[f"system_{k}_{w['n_total']}_particles"] = {
            "force_rel_rms": _rel_rms(F32[:, boff[k]:boff[k + 1]].T, ref["F"]),
            "charge_rel_rms": _rel_rms(bout["Q"][qoff[k]:qoff[k + 1]], ref["Q"]),
            "energy_rel": abs(float(bout["E"][k]) - ref["E"]) / abs(ref["E"])}
    gpath = os.path.join(GOLDEN, "uneven_largest.json")
    if os.path.exists(gpath):
        with open(gpath) as f:
            ref = json.load(f)
        k = ref["system"]
        it = items[k]
        w = systems[k]
        rs = np.random.default_rng(9)
        Qfix = w["ele_side"] * 0.004 + 0.001 * rs.normal(size=len(w["ele_side"]))
        fixed = srbe_amd.System(dict(w["params"], kspace_tol=1e-16), w["ele_pos"], w["ele_side"],
                                flags=srbe_amd.SRBE_FLAG_NO_CP)
        sdg = torch.tensor([ref["seed"]], dtype=torch.int64, device=dev).view(torch.uint64)
        o = fixed.step(it["off"], it["xyz"], it["q"], it["dp"], sdg, ref["step"], precision=srbe_amd.SRBE_FP32,
                       Q_in=torch.tensor(Qfix, dtype=torch.float64, device=dev), want_kset=False)
        torch.cuda.synchronize()
        nk = len(w["ion_q"])
        F = o["F"].cpu().numpy().reshape(3, nk)[:, ref["ion_index"]].T
        errs[f"system_{k}_{w['n_total']}_particles_sampled"] = {
            "force_rel_rms": _rel_rms(F, ref["F"]),
            "b_rel_rms": _rel_rms(o["b"].cpu().numpy()[ref["ele_index"]], ref["b"]),
            "targets": "64 ions, 64 electrodes, fixed charges (uneven_largest.json)"}
        fixed.close()
    out["fp32_error_vs_fp64_oracle"] = errs
    for it in items:
        it["sys"].close()
    return out


def count_pairs(wb, wp):
    """Ordered ion-ion pairs and ion-electrode pairs closer than rc (minimum image in x, y), summed over replicas."""
    Lx, Ly, rc2 = wp["Lx"], wp["Ly"], wp["rc"] ** 2
    ele = np.asarray(wb["ele_pos"], dtype=np.float64)

    def count(a, b, same):
        tot = 0
        for i0 in range(0, len(a), 256):
            d = a[i0:i0 + 256, None, :] - b[None, :, :]
            d[..., 0] -= Lx * np.rint(d[..., 0] / Lx)
            d[..., 1] -= Ly * np.rint(d[..., 1] / Ly)
            m = (d * d).sum(-1) < rc2
            if same:
                idx = np.arange(i0, min(i0 + 256, len(a)))
                m[idx - i0, idx] = False
            tot += int(m.sum())
        return tot

    nii = nie = 0
    for pos in wb["ion_pos"]:
        pos = np.asarray(pos, dtype=np.float64)
        nii += count(pos, pos, True)
        nie += count(pos, ele, False)
    return nii, nie


def cpu_side(wb, wp, acc, R, sizes, n_ele, K):
    """The oracle's own throughput on a bounded sample, and the FP32 errors of those replicas.

    acc: host copies of one FP32 GPU step at step index 0 (Q, F SoA, b, E, offsets).
    """
    from oracle import cp, ewald, sampler, srbe

    p = ewald.Params(Lx=wp["Lx"], Ly=wp["Ly"], H=wp["H"], lam=wp["lam"], alpha=wp["alpha"], eta=wp["eta"],
                     rc=wp["rc"], coulomb_k=wp["coulomb_k"], M=int(wp["M"]), P=int(wp["P"]),
                     kspace_tol=wp["kspace_tol"])
    t0 = time.time()
    log("building the oracle's electrode matrix ...")
    solver = cp.Solver(ewald.electrode_matrix(p, wb["ele_pos"]))
    oracle_setup_s = time.time() - t0
    log(f"oracle A in {oracle_setup_s:.1f} s; timing oracle steps")
    def oracle_steps(limit_s, count=None):
        ru0 = resource.getrusage(resource.RUSAGE_SELF)
        t0 = time.time()
        out = []
        for r in range(R if count is None else count):
            ks, _ = sampler.draw_kset(p, 2100 + r, 0, 0)
            out.append(srbe.srbe_step(p, solver, ks, wb["ion_pos"][r], wb["ion_q"][r], wb["ele_pos"],
                                      wb["ele_side"], float(wb["dpsi"][r])))
            if time.time() - t0 > limit_s:
                break
        wall = time.time() - t0
        ru1 = resource.getrusage(resource.RUSAGE_SELF)
        return out, wall, (ru1.ru_utime - ru0.ru_utime) + (ru1.ru_stime - ru0.ru_stime)

    refs, wall, cpu = oracle_steps(15.0)
    nsample = len(refs)
    pairs = sum(sizes[r] + n_ele for r in range(nsample)) * K
    # the same replicas again with every thread pool of the process limited to one thread
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        refs1, wall1, cpu1 = oracle_steps(30.0, count=nsample)
    pairs1 = sum(sizes[r] + n_ele for r in range(len(refs1))) * K
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    errs = errors_vs_oracle(refs, acc, n_ele)
    return {
        "fp32_error_vs_fp64_oracle": dict(errs, target_force_rel_rms=1e-5),
        "cpu_baseline": {"value": pairs / wall, "unit": "pairs/s", "cores": max(1, round(cpu / wall)),
                         "kind": "oracle",
                         "sample": f"FP64 numpy oracle SRBE step (sample, b*, CP solve, forces, energy) on "
                                   f"{nsample} of the {R} replicas, one step each (about 15 s); A built once "
                                   f"beforehand ({oracle_setup_s:.1f} s, not timed); cpu_time/wall = "
                                   f"{cpu / wall:.2f}; host threads available: {os.cpu_count()}",
                         "cpu_model": model, "host_threads": os.cpu_count(),
                         "one_thread": {"value": pairs1 / wall1, "unit": "pairs/s", "replicas": len(refs1),
                                        "cpu_time_over_wall": cpu1 / wall1}},
        "oracle_setup_s": oracle_setup_s,
    }, refs


def errors_vs_oracle(refs, acc, n_ele):
    """Relative errors of one GPU step (host copies in acc) against the oracle's steps refs."""
    off = acc["off"]
    N = int(off[-1])
    F = acc["F"].reshape(3, N)
    errF, errFmax, errb, errQ, errE, neut = [], [], [], [], [], []
    for r, ref in enumerate(refs):
        Fg = F[:, off[r]:off[r + 1]].T
        errF.append(np.linalg.norm(Fg - ref["F"]) / np.linalg.norm(ref["F"]))
        # worst ion's force error against the RMS force magnitude
        errFmax.append(np.max(np.linalg.norm(Fg - ref["F"], axis=1)) / np.sqrt(np.mean(np.sum(ref["F"] ** 2, axis=1))))
        bg = acc["b"][r * n_ele:(r + 1) * n_ele]
        errb.append(np.linalg.norm(bg - ref["b"]) / np.linalg.norm(ref["b"]))
        Qg = acc["Q"][r * n_ele:(r + 1) * n_ele]
        errQ.append(np.linalg.norm(Qg - ref["Q"]) / np.linalg.norm(ref["Q"]))
        neut.append(abs(np.sum(Qg)) / np.sum(np.abs(Qg)))
        errE.append(abs(acc["E"][r] - ref["E"]) / abs(ref["E"]))
    return {"force_rel_rms_max": max(errF), "force_max_ion_over_rms_max": max(errFmax), "b_rel_rms_max": max(errb),
            "charge_rel_rms_max": max(errQ), "charge_sum_over_l1_max": max(neut), "energy_rel_max": max(errE),
            "replicas_checked": len(refs)}


def error_split(srbe_amd, sysm, wb, wp, refs, off, xyz, q, dpsi, seeds, n_ele, nsplit=8):
    """FP32 force error of the k-space part, the real-space part and their sum, apart.

    Both handles run the batch at the oracle's charges (fixed-charge steps, same
    sampled modes): the k-space-only handle gives the Fourier and slab force, the
    full handle minus it the real-space force; the oracle's parts come from the same
    functions its step uses.
    """
    import torch
    from oracle import ewald, sampler, srbe

    p = ewald.Params(Lx=wp["Lx"], Ly=wp["Ly"], H=wp["H"], lam=wp["lam"], alpha=wp["alpha"], eta=wp["eta"],
                     rc=wp["rc"], coulomb_k=wp["coulomb_k"], M=int(wp["M"]), P=int(wp["P"]),
                     kspace_tol=wp["kspace_tol"])
    R = len(off) - 1
    m = min(nsplit, len(refs))
    Qh = np.zeros(R * n_ele)
    for r in range(m):
        Qh[r * n_ele:(r + 1) * n_ele] = refs[r]["Q"]
    Qin = torch.tensor(Qh, device=xyz.device)
    kso = srbe_amd.System(wp, wb["ele_pos"], wb["ele_side"],
                          flags=srbe_amd.SRBE_FLAG_NO_CP | srbe_amd.SRBE_FLAG_KSPACE_ONLY)
    full = sysm.step(off, xyz, q, dpsi, seeds, 0, precision=srbe_amd.SRBE_FP32, Q_in=Qin, want_kset=False)
    kpart = kso.step(off, xyz, q, dpsi, seeds, 0, precision=srbe_amd.SRBE_FP32, Q_in=Qin, want_kset=False)
    torch.cuda.synchronize()
    N = int(off[-1])
    Ff = full["F"].cpu().numpy().reshape(3, N)
    Fk = kpart["F"].cpu().numpy().reshape(3, N)
    kso.close()
    ek, er, et = [], [], []
    ele = np.asarray(wb["ele_pos"], dtype=np.float64)
    for r in range(m):
        ion = np.asarray(wb["ion_pos"][r], dtype=np.float64)
        qi = np.asarray(wb["ion_q"][r], dtype=np.float64)
        Q = refs[r]["Q"]
        ks, _ = sampler.draw_kset(p, 2100 + r, 0, 0)
        Fk_ref = srbe.srbe_force_fourier(p, ks, ion, qi, ele, Q)
        Fk_ref[:, 2] -= p.coulomb_k * (4.0 * np.pi / p.V) * qi * (qi @ ion[:, 2] + Q @ ele[:, 2])
        _, gii = ewald.real_space(p, "ii", ion, ion, qi, same=True)
        _, gig = ewald.real_space(p, "ig", ion, ele, Q)
        Fr_ref = -p.coulomb_k * qi[:, None] * (gii + gig)
        gk = Fk[:, off[r]:off[r + 1]].T
        gt = Ff[:, off[r]:off[r + 1]].T
        ek.append(np.linalg.norm(gk - Fk_ref) / np.linalg.norm(Fk_ref))
        er.append(np.linalg.norm((gt - gk) - Fr_ref) / np.linalg.norm(Fr_ref))
        et.append(np.linalg.norm(gt - (Fk_ref + Fr_ref)) / np.linalg.norm(Fk_ref + Fr_ref))
    return {"at_oracle_charges": {"force_rel_rms_kspace_max": max(ek), "force_rel_rms_real_space_max": max(er),
                                  "force_rel_rms_total_max": max(et), "replicas": m}}


if __name__ == "__main__":
    main()
