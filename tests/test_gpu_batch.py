"""Batches of systems of different geometry (srbe_batch_*): one launch per phase for all.

Four systems: the tiny slab (dense charge solve; two replicas of different sizes), two
small systems of the uneven batch (square-lattice walls, lattice charge solve; aspect
ratios 12 and 12, one and two replicas) and its largest system (162,990 particles: the
multi-block cell sort, the energy's tiled ion sums; one replica).  The batch step runs
the same kernels as a single-system srbe_step, so its outputs must equal those of one
srbe_step per system with the same seeds and step index: FP64 to 1e-13 relative
max-norm; FP32 to the FP32 tolerances (the batch sizes some grids from the whole batch,
which reorders FP32 sums).  The tiny slab's replicas and the smallest uneven system are
also compared with the FP64 oracle (tolerances of test_gpu_step.py).  A captured batch
step replays to the eager step's results; fixed-charge batch steps match single ones.
"""

import numpy as np
import pytest

from helpers import forces_from_soa, oracle_params, oracle_solver, oracle_step, rel_inf, rel_rms

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

STEP = 3
UNEVEN = [10, 7, 26]  # two of the smallest systems and the largest one


@pytest.fixture(scope="module")
def batch():
    import paper_2509_24742_amd as srbe_amd
    from paper_2509_24742_amd import binding
    from paper_2509_24742_amd import workloads as wl
    t0 = wl.tiny_slab(seed=1000)
    t1 = wl.tiny_slab(seed=1001)
    t1_pos, t1_q = t1["ion_pos"][:160], t1["ion_q"][:160].copy()
    t1_q -= t1_q.mean()  # a smaller, still neutral replica
    uv = wl.uneven_batch(place=set(UNEVEN))
    assert max(uv[k]["n_total"] for k in UNEVEN) > 150000
    systems = [srbe_amd.System(dict(t0["params"], kspace_tol=1e-16), t0["ele_pos"], t0["ele_side"])]
    for k in UNEVEN:
        w = uv[k]
        systems.append(srbe_amd.System(dict(w["params"], kspace_tol=1e-16), w["ele_pos"], w["ele_side"],
                                       flags=srbe_amd.SRBE_FLAG_LATTICE_SOLVE))
    # replicas: (system, positions, charges, dpsi, seed)
    reps = [(0, t0["ion_pos"], t0["ion_q"], 2.0, 2000), (0, t1_pos, t1_q, 1.0, 2001),
            (1, uv[10]["ion_pos"], uv[10]["ion_q"], 2.0, 4110),
            (2, uv[7]["ion_pos"], uv[7]["ion_q"], 1.5, 4107), (2, uv[7]["ion_pos"], uv[7]["ion_q"], 3.0, 4207),
            (3, uv[26]["ion_pos"], uv[26]["ion_q"], 2.0, 4126)]
    bt = binding.srbe_batch_create([s.h for s in systems])
    yield dict(systems=systems, reps=reps, bt=bt, t0=t0, t1=(t1_pos, t1_q), uv=uv)
    binding.srbe_batch_destroy(bt)
    for s in systems:
        s.close()


def _inputs(reps):
    dev = torch.device("cuda")
    sizes = [len(r[2]) for r in reps]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    pos = np.concatenate([np.asarray(r[1], dtype=np.float64) for r in reps])
    xyz = torch.tensor(np.ascontiguousarray(pos.T).ravel(), dtype=torch.float64, device=dev)
    q = torch.tensor(np.concatenate([r[2] for r in reps]), dtype=torch.float64, device=dev)
    dp = torch.tensor([r[3] for r in reps], dtype=torch.float64, device=dev)
    sd = torch.tensor(np.array([r[4] for r in reps], dtype=np.int64), device=dev).view(torch.uint64)
    sor = np.array([r[0] for r in reps], dtype=np.int32)
    return off, sor, xyz, q, dp, sd


def _run_batch(batch, precision, Q_in=None, graph=False):
    from paper_2509_24742_amd import binding
    off, sor, xyz, q, dp, sd = _inputs(batch["reps"])
    nq = sum(batch["systems"][k].n_ele for k in sor)
    dev = xyz.device
    R, N = len(sor), int(off[-1])
    out = dict(Q=torch.full((nq,), np.nan, dtype=torch.float64, device=dev),
               F=torch.full((3 * N,), np.nan, dtype=torch.float64, device=dev),
               b=torch.full((nq,), np.nan, dtype=torch.float64, device=dev),
               psibar=torch.full((R,), np.nan, dtype=torch.float64, device=dev),
               E=torch.full((R,), np.nan, dtype=torch.float64, device=dev))
    if graph:
        gr = binding.srbe_batch_graph_create(batch["bt"], precision, off, sor, xyz, q, dp, sd, STEP, out["Q"], out["F"],
                                             out["psibar"], Q_in=Q_in, b_out=out["b"], energy_out=out["E"])
        for _ in range(2):  # the second replay (step STEP + 1) is overwritten by the third
            binding.srbe_batch_graph_launch(gr)
        binding.srbe_batch_graph_set_step(gr, STEP)
        binding.srbe_batch_graph_launch(gr)
        torch.cuda.synchronize()
        binding.srbe_batch_graph_destroy(gr)
    else:
        binding.srbe_batch_step(batch["bt"], precision, off, sor, xyz, q, dp, sd, STEP, out["Q"], out["F"],
                                out["psibar"], Q_in=Q_in, b_out=out["b"], energy_out=out["E"])
    torch.cuda.synchronize()
    assert binding.srbe_batch_sync_status(batch["bt"]) == 0, binding.srbe_batch_last_error(batch["bt"])
    return off, sor, {k: v.cpu().numpy() for k, v in out.items()}


def _run_single(batch, precision, Q_in_list=None):
    """One srbe_step per replica on its system's handle; outputs in the batch's layout."""
    from helpers import gpu_inputs
    res = []
    for i, (k, pos, qq, dpsi, seed) in enumerate(batch["reps"]):
        off, xyz, q, dp, sd = gpu_inputs([pos], [qq], [dpsi], [seed])
        Q_in = None if Q_in_list is None else Q_in_list[i]
        out = batch["systems"][k].step(off, xyz, q, dp, sd, STEP, precision=precision, Q_in=Q_in)
        torch.cuda.synchronize()
        res.append({key: v.cpu().numpy() for key, v in out.items() if v is not None})
    return res


def _split(batch, off, sor, got, r):
    """Replica r's outputs of a batch step."""
    n = [batch["systems"][k].n_ele for k in sor]
    q0 = int(sum(n[:r]))
    N = int(off[-1])
    F = got["F"].reshape(3, N)[:, off[r]:off[r + 1]].T
    return dict(Q=got["Q"][q0:q0 + n[r]], b=got["b"][q0:q0 + n[r]], F=F, psibar=got["psibar"][r], E=got["E"][r])


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_equals_single_system_steps(batch, precision):
    """FP64: equal to 1e-13 (the sums' order aside, the same arithmetic).  FP32: a batch
    sizes the real-space work splits and the structure-factor chunks from the whole batch,
    so its FP32 sums run in another order than a lone system's; the two then agree to the
    FP32 tolerances against the oracle (force 1e-5 relative RMS, Q and b 3e-5), psibar to
    that tolerance on b (it takes up the uniform part of b's rounding, which Q does not
    see), and the energy to 1e-4 of its magnitude (it is assembled from terms some 30 times
    its size, each good to a few 1e-7 relative)."""
    off, sor, got = _run_batch(batch, precision)
    ref = _run_single(batch, precision)
    same = True
    for r in range(len(sor)):
        g = _split(batch, off, sor, got, r)
        s = ref[r]
        F1 = s["F"].reshape(3, -1).T
        same &= bool(np.array_equal(g["F"], F1) and np.array_equal(g["Q"], s["Q"]))
        dpsi_bar = abs(g["psibar"] - s["psibar"][0])
        dE = abs(g["E"] - s["E"][0])
        print(f"precision {precision} replica {r} (system {sor[r]}): F {rel_rms(g['F'], F1):.1e}, "
              f"Q {rel_inf(g['Q'], s['Q']):.1e}, b {rel_rms(g['b'], s['b']):.1e}, psibar {dpsi_bar:.1e} "
              f"(max |b| {np.abs(s['b']).max():.2f}), E {dE:.1e} of {abs(s['E'][0]):.2f}", flush=True)
        if precision == 0:
            tol = 1e-13
            assert rel_rms(g["F"], F1) <= tol and rel_inf(g["F"], F1) <= 100 * tol
            assert rel_inf(g["Q"], s["Q"]) <= 10 * tol and rel_inf(g["b"], s["b"]) <= 10 * tol
            assert dpsi_bar <= 10 * tol * max(1.0, abs(s["psibar"][0]))
            assert dE <= 10 * tol * abs(s["E"][0])
        else:
            assert rel_rms(g["F"], F1) <= 1e-5
            assert rel_rms(g["Q"], s["Q"]) <= 3e-5 and rel_rms(g["b"], s["b"]) <= 3e-5
            assert dpsi_bar <= 3e-5 * np.abs(s["b"]).max()
            assert dE <= 1e-4 * abs(s["E"][0])
    print(f"precision {precision}: bitwise equal to the single-system steps: {same}", flush=True)


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_matches_oracle(batch, precision):
    off, sor, got = _run_batch(batch, precision)
    t0, (t1_pos, t1_q), uv = batch["t0"], batch["t1"], batch["uv"]
    cases = [(0, t0["params"], t0["ion_pos"], t0["ion_q"], t0["ele_pos"], t0["ele_side"]),
             (1, t0["params"], t1_pos, t1_q, t0["ele_pos"], t0["ele_side"]),
             (2, uv[10]["params"], uv[10]["ion_pos"], uv[10]["ion_q"], uv[10]["ele_pos"], uv[10]["ele_side"])]
    solvers = {}
    for r, params, pos, qq, ele, side in cases:
        p = oracle_params(dict(params, kspace_tol=1e-16))
        key = id(params)
        if key not in solvers:
            solvers[key] = oracle_solver(p, ele)
        _, _, _, dpsi, seed = batch["reps"][r]
        ref = oracle_step(p, solvers[key], seed, STEP, pos, qq, ele, side, dpsi)
        g = _split(batch, off, sor, got, r)
        print(f"precision {precision} replica {r}: F {rel_rms(g['F'], ref['F']):.2e}, Q {rel_inf(g['Q'], ref['Q']):.2e}",
              flush=True)
        if precision == 0:
            assert rel_inf(g["F"], ref["F"]) < 1e-11 and rel_inf(g["Q"], ref["Q"]) < 1e-11
            assert rel_inf(g["b"], ref["b"]) < 1e-11
            assert abs(g["E"] - ref["E"]) < 1e-11 * abs(ref["E"])
            assert abs(g["psibar"] - ref["psibar"]) < 1e-11 * max(1.0, abs(ref["psibar"]))
        else:
            assert rel_rms(g["F"], ref["F"]) < 1e-5
            assert rel_rms(g["Q"], ref["Q"]) < 3e-5 and rel_rms(g["b"], ref["b"]) < 3e-5


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_graph_replay_equals_eager(batch, precision):
    off, sor, eager = _run_batch(batch, precision)
    _, _, replay = _run_batch(batch, precision, graph=True)
    for key in eager:
        assert np.array_equal(eager[key], replay[key]), key


def test_batch_fixed_charges(batch):
    off, sor, _ = _run_batch(batch, 0)
    rng = np.random.default_rng(5)
    n = [batch["systems"][k].n_ele for k in sor]
    Qs = [rng.normal(size=m) * 0.01 for m in n]
    dev = torch.device("cuda")
    Q_in = torch.tensor(np.concatenate(Qs), dtype=torch.float64, device=dev)
    _, _, got = _run_batch(batch, 1, Q_in=Q_in)
    ref = _run_single(batch, 1, [torch.tensor(q, dtype=torch.float64, device=dev) for q in Qs])
    for r in range(len(sor)):
        g = _split(batch, off, sor, got, r)
        F1 = ref[r]["F"].reshape(3, -1).T
        assert rel_rms(g["F"], F1) <= 1e-6
        assert np.array_equal(g["Q"], Qs[r])
        assert np.isnan(g["psibar"]) and np.isnan(g["E"])


def test_batch_rejects_bad_arguments(batch):
    from paper_2509_24742_amd import binding
    off, sor, xyz, q, dp, sd = _inputs(batch["reps"])
    nq = sum(batch["systems"][k].n_ele for k in sor)
    dev = xyz.device
    Q = torch.empty(nq, dtype=torch.float64, device=dev)
    F = torch.empty(3 * int(off[-1]), dtype=torch.float64, device=dev)
    ps = torch.empty(len(sor), dtype=torch.float64, device=dev)
    bad = sor.copy()
    bad[0], bad[-1] = bad[-1], bad[0]  # not grouped by system
    with pytest.raises(binding.SrbeError) as ei:
        binding.srbe_batch_step(batch["bt"], 0, off, bad, xyz, q, dp, sd, 0, Q, F, ps)
    assert ei.value.code == binding.SRBE_EINVAL
    assert "non-decreasing" in binding.srbe_batch_last_error(batch["bt"])
