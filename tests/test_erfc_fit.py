"""The FP32 erfc used by the real-space pair kernels (coefficients read from the kernel source)
against scipy's scaled complementary error function, evaluated in FP32 as on the GPU."""
import os
import re

import numpy as np
from scipy.special import erfc, erfcx

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2011_01207_amd", "csrc",
                   "realspace.hip")


def kernel_coefficients():
    body = open(SRC).read()
    body = body[body.index("d_erfc_g(float x, float gauss)"):]
    body = body[:body.index("return p * gauss;")]
    first = float(re.search(r"float p = ([-0-9.e+]+)f;", body).group(1))
    rest = [float(v) for v in re.findall(r"fmaf\(p, t, ([-0-9.e+]+)f\)", body)]
    return [first] + rest   # highest order first


def test_fp32_erfc_relative_error():
    coef = np.array(kernel_coefficients(), dtype=np.float32)
    assert len(coef) == 10
    x = np.linspace(0.0, 4.5, 200001).astype(np.float32)
    t0 = (np.float32(1.0) / (np.float32(1.0) + np.float32(0.5) * x)).astype(np.float32)
    # the kernel takes t from the hardware reciprocal (within 1 ulp): check t and its neighbours
    for t in (t0, np.nextafter(t0, np.float32(0.0)), np.nextafter(t0, np.float32(2.0))):
        p = np.full_like(t, coef[0])
        for cval in coef[1:]:
            p = (p * t + cval).astype(np.float32)
        rel = np.abs(p.astype(np.float64) - erfcx(x.astype(np.float64))) / erfcx(x.astype(np.float64))
        assert rel.max() < 6e-7
        # with the Gaussian factor: erfc itself to FP32-level relative accuracy
        e = p.astype(np.float64) * np.exp(-x.astype(np.float64) ** 2)
        assert np.max(np.abs(e - erfc(x.astype(np.float64))) / erfc(x.astype(np.float64))) < 6e-7
