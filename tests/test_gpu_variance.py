"""The SRBE estimator's spread at a fixed configuration (Remark 3.1), measured on the GPU.

One step of 256 replicas of the tiny slab with 256 seeds draws 256 independent samples
of the charge on the negative electrode.  Checked: (1) the deterministic kz modes cut
the charge's standard deviation (M = 10, the aspect ratio, against M = 0, at P = 50),
(2) four times the batch size roughly halves it (P = 200 against P = 50, at M = 10),
and (3) the sample mean is the oracle's complete-Ewald charge (Theorems 3.1, 3.2:
the estimator is unbiased) within four standard errors.
"""

import numpy as np
import pytest

from helpers import oracle_params, oracle_solver

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SAMPLES = 256


@pytest.fixture(scope="module")
def runs():
    from paper_2509_24742_amd import variance_study as vs
    w, _ = vs.configuration("tiny")
    out = {}
    for M, P in [(0, 50), (10, 50), (10, 200)]:
        Q, F = vs.sample_step(w, M, P, SAMPLES)
        out[(M, P)] = vs.statistics(w, Q, F)
        print(f"M {M} P {P}: {out[(M, P)]}", flush=True)
    return w, out


def test_deterministic_modes_cut_the_charge_spread(runs):
    _, s = runs
    assert s[(10, 50)]["q_neg_sd"] < 0.5 * s[(0, 50)]["q_neg_sd"]


def test_batch_size_reduces_the_spread(runs):
    _, s = runs
    ratio = s[(10, 200)]["q_neg_sd"] / s[(10, 50)]["q_neg_sd"]
    assert 0.3 < ratio < 0.75  # 1/sqrt(4) = 0.5 up to the sampling error of two SDs of 256 samples
    assert s[(10, 200)]["force_rel_sd"] < s[(10, 50)]["force_rel_sd"]


def test_mean_charge_is_the_complete_ewald_charge(runs):
    from oracle import srbe
    w, s = runs
    p = oracle_params(dict(w["params"], kspace_tol=1e-16))
    ref = srbe.full_step(p, oracle_solver(p, w["ele_pos"]), w["ion_pos"], w["ion_q"], w["ele_pos"], w["ele_side"], 2.0)
    q_exact = float(np.sum(ref["Q"][np.asarray(w["ele_side"]) < 0]))
    st = s[(10, 200)]
    se = st["q_neg_sd"] / np.sqrt(SAMPLES)
    print(f"exact {q_exact:.6f}, sample mean {st['q_neg_mean']:.6f} +- {se:.6f}", flush=True)
    assert abs(st["q_neg_mean"] - q_exact) < 4 * se
