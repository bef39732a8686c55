"""The branch-free FP32 erfc of the mixed-precision Ewald real-space sum
(common.hpp): its coefficients, read from the header, reproduce erfc to the fit's
accuracy in FP64 and to FP32 rounding in an FP32 emulation."""
import os
import re

import numpy as np
from scipy.special import erfc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _coeffs():
    src = open(os.path.join(ROOT, "paper_1605_08423_amd", "csrc", "common.hpp")).read()
    body = src[src.index("dev_erfc_exp<float>(float x"):]
    q = dict((int(k), float(v)) for k, v in re.findall(r"Q(\d) = (-?[0-9.e-]+)f", body))
    p = float(re.search(r"fmaf\(([0-9.]+)f, x, 1.0f\)", body).group(1))
    return p, np.array([q[k] for k in range(len(q))])


def _approx(x, p, c, dt):
    x = x.astype(dt)
    t = (dt(1) / (dt(1) + dt(p) * x)).astype(dt)
    q = np.zeros_like(t)
    for a in c[::-1].astype(dt):
        q = (q * t + a).astype(dt)
    hi = (x * x).astype(dt)
    lo = (x.astype(np.float64) ** 2 - hi.astype(np.float64)).astype(dt)
    e = (np.exp(-hi).astype(dt) * (dt(1) - lo)).astype(dt)
    return (t * q * e).astype(dt)


def test_fit_accuracy_fp64():
    p, c = _coeffs()
    assert len(c) == 10 and p == 0.4
    x = np.linspace(0.0, 10.0, 100001)
    rel = np.abs(_approx(x, p, c, np.float64) / erfc(x) - 1.0)
    assert rel.max() < 5e-8          # fit 8e-9 plus rounding the coefficients to FP32


def test_fp32_emulation_absolute_error():
    p, c = _coeffs()
    x = np.linspace(0.0, 8.0, 200001)
    v = _approx(x, p, c, np.float32).astype(np.float64)
    ref = erfc(x)
    # three rounded products, the polynomial and e^{-x^2} in FP32: a few ulp (measured
    # 3.6e-7 absolute near x = 0, 1.1e-6 relative where erfc ~ 1e-6)
    big = ref > 1e-6
    assert np.abs(v[big] / ref[big] - 1.0).max() < 2e-6
    assert np.abs(v - ref).max() < 5e-7
