"""Generate the FP32 erfc coefficients of the real-space pair kernels (realspace.hip).

erfc(x) = P(t) exp(-x^2) with t = 1 / (1 + x/2), P a degree-9 polynomial fitted to the scaled
complementary error function erfc(x) exp(x^2) on x in [0, 4.5] (beta * cutoff is 3.8 for the
workloads here) by least squares on a Chebyshev grid in t, reweighted towards minimax relative
error.  Run: python fit_erfc.py  (prints the coefficients, lowest order first)."""
import numpy as np
from scipy.special import erfcx

P_SCALE, DEG, XMAX = 0.5, 9, 4.5


def fit():
    tmin = 1.0 / (1.0 + P_SCALE * XMAX)
    t = np.cos(np.linspace(0, np.pi, 4000)) * (1 - tmin) / 2 + (1 + tmin) / 2
    x = (1 / t - 1) / P_SCALE
    f = erfcx(x)
    V = np.vander(t, DEG + 1, increasing=True)
    w = 1 / f
    c, *_ = np.linalg.lstsq(V * w[:, None], f * w, rcond=None)
    for _ in range(30):
        r = np.abs(V @ c - f) / f
        w2 = w * (1 + 50 * r / r.max())
        c, *_ = np.linalg.lstsq(V * w2[:, None], f * w2, rcond=None)
    return c


if __name__ == "__main__":
    for k, v in enumerate(fit()):
        print(f"c{k} = {v:.9e}")
