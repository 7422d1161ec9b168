"""Coefficients of the FP32 erfc used by the real-space kernels.

    python paper_2509_24742_amd/csrc/fit_erfc.py

The scaled complementary error function erfcx(x) = exp(x^2) erfc(x) is smooth and
bounded on x >= 0; with t = 1 / (1 + x / 2) (which maps [0, inf) onto (0, 1]) it is
written as t p(t) with p a polynomial of degree 9.  The coefficients come from a
near-minimax fit of the relative error on x in [0, 10] (Lawson's iteratively
reweighted least squares); beyond x = 10, erfc is below the smallest FP32 normal.
Printed: the coefficients rounded to FP32, the fitted relative error in FP64 and the
error of the FP32 evaluation (t by a correctly rounded reciprocal, Horner in FP32).
"""

import numpy as np
from scipy.special import erfcx

DEG = 9
C = 0.5
XMAX = 10.0


def fit():
    x = np.linspace(0.0, XMAX, 200001)
    t = 1.0 / (1.0 + C * x)
    y = erfcx(x) / t
    V = np.vander(t, DEG + 1, increasing=True)
    w = 1.0 / y
    wt = np.ones_like(x)
    for _ in range(80):
        sw = np.sqrt(wt)
        coef, *_ = np.linalg.lstsq(V * (w * sw)[:, None], y * w * sw, rcond=None)
        err = (V @ coef - y) / y
        wt = wt * np.abs(err)
        wt /= wt.mean()
    return coef, np.max(np.abs(err))


def eval32(coef, x):
    cf = coef.astype(np.float32)
    t = (np.float32(1) / (np.float32(1) + np.float32(C) * x.astype(np.float32))).astype(np.float32)
    p = np.full_like(t, cf[-1])
    for a in cf[-2::-1]:
        p = (p * t + a).astype(np.float32)
    return (t * p).astype(np.float64)


if __name__ == "__main__":
    coef, e64 = fit()
    x = np.linspace(0.0, XMAX, 400001)
    e32 = np.max(np.abs(eval32(coef, x) / erfcx(x) - 1))
    print("// p(t), t = 1/(1 + x/2); rel. err. of t p(t): %.2e (FP64 fit), %.2e (FP32 evaluation)" % (e64, e32))
    print(", ".join("%.9ef" % np.float32(c) for c in coef))
