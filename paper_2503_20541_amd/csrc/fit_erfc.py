"""Coefficients of the pair kernel's scaled complementary error function.

The real-space Ewald term needs erfc(x) for x = alpha r. The kernel evaluates
erfc(x) = exp(-x^2) R(x) with R(x) = exp(x^2) erfc(x) approximated as t P(t),
t = 1 / (1 + p x), P a polynomial of degree 7 (the exp(-x^2) factor is needed
for the force anyway). This script fits P by weighted least squares on the
relative error over x in [0, 6], reweighting towards equal ripple, for a grid
of p, and prints the best p and P's coefficients (highest degree first, in
the order the kernel's Horner scheme uses them) with the maximum relative
error on a dense grid. Run it with numpy and scipy:

    python paper_2503_20541_amd/csrc/fit_erfc.py
"""
import numpy as np
from scipy.special import erfcx

DEGREE = 7
X_MAX = 6.0


def fit(p, deg=DEGREE, x_max=X_MAX, iters=40):
    x = np.linspace(0.0, x_max, 40001)
    t = 1.0 / (1.0 + p * x)
    r = erfcx(x)
    a = np.vander(t, deg + 1, increasing=True) * t[:, None]
    w = np.ones_like(x)
    for _ in range(iters):
        c, *_ = np.linalg.lstsq(a * (w / r)[:, None], w, rcond=None)
        err = (a @ c) / r - 1.0
        w = w * (1.0 + 5.0 * np.abs(err) / np.abs(err).max())
    err = (a @ c) / r - 1.0
    return c, float(np.abs(err).max())


def float32_error(p, c, x_max=X_MAX):
    """Max relative error of the float32 Horner evaluation the kernel does."""
    x = np.linspace(0.0, x_max, 200001).astype(np.float32)
    t = (np.float32(1.0) / (np.float32(p) * x + np.float32(1.0))).astype(np.float32)
    q = np.float32(c[-1])
    for k in range(len(c) - 2, -1, -1):
        q = (q * t + np.float32(c[k])).astype(np.float32)
    val = (q * t).astype(np.float64)
    return float(np.abs(val / erfcx(x.astype(np.float64)) - 1.0).max())


if __name__ == "__main__":
    best = None
    for p in np.round(np.arange(0.20, 0.80001, 0.005), 3):
        c, e = fit(p)
        if best is None or e < best[1]:
            best = (c, e, p)
    c, e, p = best
    print(f"p = {p:.3f}f; max relative error {e:.2e} (exact arithmetic), "
          f"{float32_error(p, c):.2e} (float32 evaluation)")
    for k in range(len(c) - 1, -1, -1):
        print(f"  c{k} = {np.float32(c[k]):.9e}f")
