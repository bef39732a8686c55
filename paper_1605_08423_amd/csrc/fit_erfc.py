"""Fits the coefficients of the branch-free FP32 erfc in common.hpp.

erfc(x) = t Q(t) exp(-x^2) with t = 1 / (1 + P x) for x >= 0, so Q(t) = erfcx(x) / t
is smooth on t in (0, 1].  Q is a degree-9 polynomial from weighted least squares
in relative error on x in [0, 10], reweighted toward equal ripple (Lawson's
iteration).  Reference values are scipy.special.erfcx.  Prints the C literals.
"""
import numpy as np
from scipy.special import erfcx

P, DEG, XMAX = 0.4, 9, 10.0


def fit(p=P, deg=DEG, xmax=XMAX, iters=30):
    xs = np.linspace(0.0, xmax, 200001)
    t = 1.0 / (1.0 + p * xs)
    y = erfcx(xs) / t
    V = np.vander(t, deg + 1, increasing=True)
    w = np.ones_like(xs)
    for _ in range(iters):
        c, *_ = np.linalg.lstsq(V / y[:, None] * w[:, None], w, rcond=None)
        rel = (V @ c) / y - 1.0
        w = w * (np.abs(rel) / np.abs(rel).max()) ** 0.5 + 1e-12
        w /= w.max()
    rel = (V @ c) / y - 1.0
    return c, float(np.abs(rel).max())


if __name__ == "__main__":
    c, err = fit()
    print(f"// P = {P}, degree {DEG}, max relative error of the fit {err:.2e}")
    for k, v in enumerate(c):
        print(f"  constexpr float Q{k} = {np.float32(v)!r}f;".replace("np.float32(", "").replace(")f", "f"))
