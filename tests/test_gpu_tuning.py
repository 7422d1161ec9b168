"""Launch parameters (srbe_get_tuning / srbe_set_tuning, the cache of choices) through the C ABI.

Every tunable launch shape must give the oracle's results: each setting below is run
on a three-replica batch of the tiny slab and compared with the FP64 oracle on the
same sample, to the tolerances of test_gpu_step.py (FP64: 1e-11 relative max-norm;
FP32: force relative RMS <= 1e-5, b and Q <= 3e-5).  The settings cover every value
of the waves-per-block, unroll, electrode-split and GEMM-depth parameters, GEMM
splits from 1 to the maximum of 16 (with 32-k blocks, more ranges than blocks for
the tiny cell: some ranges are empty), and extreme chunk and real-space sizes (one
ion per wave, one block per replica, more blocks than work).
"""

import numpy as np
import pytest

from helpers import forces_from_soa, gpu_inputs, oracle_params, oracle_solver, oracle_step, rel_inf, rel_rms

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SEEDS = [2000, 31, 77]
DPSI = [1.0, 0.5, 2.0]
STEP = 5


@pytest.fixture(scope="module")
def batch():
    import paper_2509_24742_amd as srbe_amd
    from paper_2509_24742_amd import workloads as wl
    w = wl.tiny_slab()
    wp = dict(w["params"], kspace_tol=1e-16)
    p = oracle_params(wp)
    solver = oracle_solver(p, w["ele_pos"])
    sysm = srbe_amd.System(wp, w["ele_pos"], w["ele_side"])
    refs = [oracle_step(p, solver, s, STEP, w["ion_pos"], w["ion_q"], w["ele_pos"], w["ele_side"], d)
            for s, d in zip(SEEDS, DPSI)]
    reps = [w["ion_pos"]] * 3, [w["ion_q"]] * 3
    inputs = gpu_inputs(reps[0], reps[1], DPSI, SEEDS)
    yield dict(w=w, sys=sysm, refs=refs, inputs=inputs)
    sysm.close()


def run(batch, precision):
    from paper_2509_24742_amd import binding
    off, xyz, q, dp, sd = batch["inputs"]
    out = batch["sys"].step(off, xyz, q, dp, sd, STEP, precision=precision)
    torch.cuda.synchronize()
    assert binding.srbe_sync_status(batch["sys"].h) == 0, binding.srbe_last_error(batch["sys"].h)
    return off, out


def check(batch, precision, off, out, label):
    n = batch["sys"].n_ele
    for r, ref in enumerate(batch["refs"]):
        F = forces_from_soa(out["F"], off, r)
        b = out["b"].cpu().numpy()[r * n:(r + 1) * n]
        Q = out["Q"].cpu().numpy()[r * n:(r + 1) * n]
        if precision == 0:
            assert rel_inf(F, ref["F"]) < 1e-11, (label, r)
            assert rel_inf(b, ref["b"]) < 1e-11, (label, r)
            assert rel_inf(Q, ref["Q"]) < 1e-11, (label, r)
            assert abs(float(out["E"][r]) - ref["E"]) < 1e-11 * abs(ref["E"]), (label, r)
        else:
            assert rel_rms(F, ref["F"]) < 1e-5, (label, r)
            assert rel_rms(b, ref["b"]) < 3e-5 and rel_rms(Q, ref["Q"]) < 3e-5, (label, r)


LIVE_TIMING_OFF = pytest.mark.skip(reason="srbe_tune live timing is switched off: processes that ran it "
                                   "aborted (host heap corruption, cause not found)")


# sf_blocks, waves, unroll, ii_ions, ie_blocks, ele_split, gemm_split, gemm_depth
SETTINGS = [
    [256, 2, 2, 1, 1, 1, 1, 2],
    [4096, 8, 8, 7, 3, 4, 16, 2],
    [512, 4, 8, 2, 9, 2, 3, 1],
    [2048, 2, 4, 40, 64, 1, 7, 1],
    [100, 8, 2, 3, 2, 2, 15, 2],
    [1, 4, 4, 1024, 65536, 4, 2, 2],
]


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("setting", range(len(SETTINGS)))
def test_every_setting_matches_oracle(batch, precision, setting):
    from paper_2509_24742_amd import binding
    off = batch["inputs"][0]
    h = batch["sys"].h
    binding.srbe_set_tuning(h, precision, off, SETTINGS[setting])
    try:
        assert binding.srbe_get_tuning(h, precision, off) == SETTINGS[setting]
        off_, out = run(batch, precision)
        print(f"precision {precision} setting {SETTINGS[setting]}", flush=True)
        check(batch, precision, off_, out, SETTINGS[setting])
    finally:
        binding.srbe_set_tuning(h, precision, off, None)


def test_bad_settings_rejected(batch):
    from paper_2509_24742_amd import binding
    off = batch["inputs"][0]
    h = batch["sys"].h
    base = list(binding.srbe_get_tuning(h, 1, off))
    for k, v in [(0, 0), (1, 3), (1, 16), (2, 1), (2, 16), (3, 0), (4, 0), (5, 3), (5, 8), (6, 0), (6, 17), (7, 0), (7, 3)]:
        bad = list(base)
        bad[k] = v
        with pytest.raises(binding.SrbeError) as ei:
            binding.srbe_set_tuning(h, 1, off, bad)
        assert ei.value.code == binding.SRBE_EINVAL
    assert binding.srbe_get_tuning(h, 1, off) == base  # nothing stored


def test_live_timing_is_switched_off(batch):
    # srbe_tune's live timing is switched off (processes that ran it have aborted with
    # host heap corruption of unknown cause): it returns SRBE_EINVAL with a message
    # and stores nothing
    from paper_2509_24742_amd import binding
    off, xyz, q, dp, sd = batch["inputs"]
    h = batch["sys"].h
    defaults = binding.srbe_get_tuning(h, 1, off)
    with pytest.raises(binding.SrbeError) as ei:
        binding.srbe_tune(h, 1, off, xyz, q, dp, sd, iters=3)
    assert ei.value.code == binding.SRBE_EINVAL
    assert "switched off" in binding.srbe_last_error(h)
    assert binding.srbe_get_tuning(h, 1, off) == defaults


@LIVE_TIMING_OFF
@pytest.mark.parametrize("precision", [0, 1])
def test_tune_stores_a_valid_choice(batch, precision):
    from paper_2509_24742_amd import binding
    off, xyz, q, dp, sd = batch["inputs"]
    h = batch["sys"].h
    defaults = binding.srbe_get_tuning(h, precision, off)
    params, ms0, ms1 = binding.srbe_tune(h, precision, off, xyz, q, dp, sd, iters=3)
    print(f"precision {precision}: defaults {defaults} ({ms0:.4f} ms) -> {params} ({ms1:.4f} ms)", flush=True)
    assert ms0 > 0 and 0 < ms1 <= ms0
    assert binding.srbe_get_tuning(h, precision, off) == params
    binding.srbe_set_tuning(h, precision, off, params)  # a valid setting
    off_, out = run(batch, precision)
    check(batch, precision, off_, out, params)
    binding.srbe_set_tuning(h, precision, off, None)
    assert binding.srbe_get_tuning(h, precision, off) == defaults


@LIVE_TIMING_OFF
def test_tune_cache_round_trip(batch, tmp_path):
    from paper_2509_24742_amd import binding
    off, xyz, q, dp, sd = batch["inputs"]
    sysm = batch["sys"]
    path = str(tmp_path / "tuning.json")
    first = sysm.tune(off, xyz, q, dp, sd, precision=1, iters=2, cache=path)
    assert not first["cached"]
    binding.srbe_set_tuning(sysm.h, 1, off, None)
    second = sysm.tune(off, xyz, q, dp, sd, precision=1, iters=2, cache=path)
    assert second["cached"] and second["params"] == first["params"]
    assert binding.srbe_get_tuning(sysm.h, 1, off) == first["params"]
    binding.srbe_set_tuning(sysm.h, 1, off, None)


@pytest.mark.parametrize("precision", [0, 1])
def test_cache_hit_applies_stored_choice(batch, precision, tmp_path):
    # a cache entry for this shape is applied without timing, and the step it gives
    # matches the oracle; a miss with tune_missing false keeps the defaults and
    # writes nothing
    import json
    import torch as _torch
    from paper_2509_24742_amd import SRBE_TUNE_NAMES, binding
    off, xyz, q, dp, sd = batch["inputs"]
    sysm = batch["sys"]
    arch = _torch.cuda.get_device_properties(dp.device).gcnArchName
    key = (f"{arch}|{'fp32' if precision else 'fp64'}|R={len(off) - 1}|maxrep={int(np.diff(off).max())}|"
           f"n_ele={sysm.n_ele}|P={sysm.params['P']}")
    chosen = SETTINGS[1]
    path = tmp_path / "tuning.json"
    path.write_text(json.dumps({key: dict(params=dict(zip(SRBE_TUNE_NAMES, chosen)), ms_default=None,
                                          ms_tuned=None)}))
    try:
        hit = sysm.tune(off, xyz, q, dp, sd, precision=precision, cache=str(path))
        assert hit["cached"] and hit["params"] == chosen
        assert binding.srbe_get_tuning(sysm.h, precision, off) == chosen
        off_, out = run(batch, precision)
        check(batch, precision, off_, out, chosen)
    finally:
        binding.srbe_set_tuning(sysm.h, precision, off, None)
    defaults = binding.srbe_get_tuning(sysm.h, precision, off)
    miss = tmp_path / "empty.json"
    got = sysm.tune(off, xyz, q, dp, sd, precision=precision, cache=str(miss), tune_missing=False)
    assert not got["cached"] and got["params"] == defaults and not miss.exists()
