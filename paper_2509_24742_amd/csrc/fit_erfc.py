"""Coefficients of the FP32 and FP64 erfc used by the real-space kernels.

    python paper_2509_24742_amd/csrc/fit_erfc.py

The scaled complementary error function erfcx(x) = exp(x^2) erfc(x) is smooth and
bounded on x >= 0; with t = 1 / (1 + x / 2) (which maps [0, inf) onto (0, 1]) it is
written as t p(t).

FP32: p a polynomial of degree 9 in t.  The coefficients come from a near-minimax fit
of the relative error on x in [0, 10] (Lawson's iteratively reweighted least squares);
beyond x = 10, erfc is below the smallest FP32 normal.  Printed: the coefficients
rounded to FP32, the fitted relative error in FP64 and the error of the FP32
evaluation (t by a correctly rounded reciprocal, Horner in FP32).

FP64: p a polynomial of degree 20 in u = (2 t - 1 - t0) / (1 - t0), t0 = t(27), which
maps x in [0, 27] onto u in [-1, 1] (beyond x = 27, erfc is below the smallest FP64
subnormal); the same fit in the Chebyshev basis, converted to powers of u.  Printed:
the coefficients and the relative error of t p evaluated by Horner in FP64 against
scipy's erfcx (whose own error bounds what a fit can show: about 1e-14).
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


DEG64 = 20
XMAX64 = 27.0


def fit64():
    from numpy.polynomial import chebyshev as cheb
    x = np.concatenate([np.linspace(0.0, 6.0, 300001), np.linspace(6.0, XMAX64, 100001)])
    t = 1.0 / (1.0 + C * x)
    t0 = 1.0 / (1.0 + C * XMAX64)
    u = (2.0 * t - 1.0 - t0) / (1.0 - t0)
    y = erfcx(x) / t
    V = cheb.chebvander(u, DEG64)
    wt = np.ones_like(x)
    for _ in range(40):
        sw = np.sqrt(wt) / y
        c, *_ = np.linalg.lstsq(V * sw[:, None], y * sw, rcond=None)
        err = (V @ c - y) / y
        wt = wt * (np.abs(err) + 1e-30)
        wt /= wt.mean()
    pm = cheb.cheb2poly(c)
    p = np.full_like(u, pm[-1])
    for a in pm[-2::-1]:
        p = p * u + a
    return pm, t0, np.max(np.abs(p / y - 1))


if __name__ == "__main__":
    coef, e64 = fit()
    x = np.linspace(0.0, XMAX, 400001)
    e32 = np.max(np.abs(eval32(coef, x) / erfcx(x) - 1))
    print("// p(t), t = 1/(1 + x/2); rel. err. of t p(t): %.2e (FP64 fit), %.2e (FP32 evaluation)" % (e64, e32))
    print(", ".join("%.9ef" % np.float32(c) for c in coef))
    pm, t0, e = fit64()
    print("// FP64: p(u), u = (2 t - 1 - t0) / (1 - t0), t0 = %.17g; rel. err. of t p(t) (Horner, FP64): %.2e"
          % (t0, e))
    print(", ".join("%.17e" % c for c in pm))
