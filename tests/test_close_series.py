"""The short-range series of the FP32 pair kernels (coefficients read from the kernel source):
B1', B2', B3' of very close pairs evaluated as the kernel does, in FP32, against the defining
formulas (Ewald recursion from erfc, Ren-Ponder Thole damping) evaluated with 60-digit decimal
arithmetic, where the cancellation of the direct formula does not matter."""
import math
import os
import re
from decimal import Decimal, getcontext

import numpy as np
import pytest

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2011_01207_amd", "csrc",
                   "realspace.hip")


def tables():
    body = open(SRC).read()
    out = {}
    for name in ("kD1", "kD2", "kD3", "kPhi3", "kPhi5", "kPsi7"):
        m = re.search(r"constexpr double %s\[(\d+)\] = \{([^}]*)\};" % name, body)
        vals = [float(v) for v in m.group(2).replace("\n", " ").split(",")]
        assert len(vals) == int(m.group(1))
        out[name] = vals
    return out


def horner32(c, t):
    p = np.float32(c[-1])
    for ck in reversed(c[:-1]):
        p = np.float32(p * t + np.float32(ck))
    return p


def kernel_close(r, beta, a, alpha_i, alpha_j, tab):
    """The kernel's short-range branch, step by step in FP32."""
    f = np.float32
    r = f(r)
    r2 = f(r * r)
    rinv = f(f(1) / r)
    w = f(f(alpha_i ** (-1.0 / 6.0)) * f(alpha_j ** (-1.0 / 6.0)))
    be = f(beta)
    be2 = f(be * be)
    x2 = f(be2 * r2)
    be3 = f(be2 * be)
    be5 = f(be3 * be2)
    A = f(f(f(f(a) * w) * w) * w)
    eps = f(f(A * r2) * r)
    if eps < 1:
        ph3, ph5, ps7 = horner32(tab["kPhi3"], eps), horner32(tab["kPhi5"], eps), horner32(tab["kPsi7"], eps)
    else:
        ex = f(math.exp(-float(eps)))
        ie = f(f(1) / eps)
        ph3 = f(f(f(1) - ex) * ie)
        ph5 = f(f(f(f(1) - f(f(1) + eps) * ex) * ie) * ie)
        ps7 = f(f(f(f(1) - f(f(1) + eps + f(0.6) * eps * eps) * ex) * ie) * ie)
    b1p = f(be3 * horner32(tab["kD1"], x2) + A * ph3)
    b2p = f(be5 * horner32(tab["kD2"], x2) + f(3) * A * A * r * ph5)
    b3p = f(be5 * be2 * horner32(tab["kD3"], x2) + f(15) * A * A * ps7 * rinv)
    return float(b1p), float(b2p), float(b3p)


def exact(r, beta, a, alpha_i, alpha_j):
    """B1', B2', B3' from their definitions with 60 significant digits."""
    getcontext().prec = 60
    r = Decimal(r)
    beta = Decimal(beta)
    pi = Decimal("3.14159265358979323846264338327950288419716939937510582097494459")
    sqrtpi = pi.sqrt()
    x = beta * r
    # erf by its Maclaurin series (x < 1 here)
    term, erf, k = x, Decimal(0), 0
    while True:
        t = term / (2 * k + 1)
        erf += t
        if abs(t) < Decimal(10) ** -58:
            break
        k += 1
        term = -term * x * x / k
    erf *= 2 / sqrtpi
    gauss = (-(x * x)).exp()
    b = [(1 - erf) / r]
    for n in (1, 2, 3):
        b.append(((2 * n - 1) * b[-1] + (2 * beta * beta) ** n * gauss / (beta * sqrtpi)) / (r * r))
    u = r / (Decimal(alpha_i) * Decimal(alpha_j)) ** (Decimal(1) / 6)
    eps = Decimal(a) * u ** 3
    ex = (-eps).exp()
    l3 = 1 - ex
    l5 = 1 - (1 + eps) * ex
    l7 = 1 - (1 + eps + Decimal(3) / 5 * eps * eps) * ex
    b1p = b[1] - (1 - l3) / r ** 3
    b2p = b[2] - 3 * (1 - l5) / r ** 5
    b3p = b[3] - 15 * (1 - l7) / r ** 7
    return float(b1p), float(b2p), float(b3p)


@pytest.mark.parametrize("r", [1e-3, 5e-3, 0.02, 0.1, 0.25, 0.4, 0.499])
@pytest.mark.parametrize("params", [(0.545, 0.39, 0.496, 0.496), (0.545, 0.39, 0.837, 0.496), (0.9, 0.39, 1.33, 0.5),
                                    (0.545, 1.0, 0.05, 0.05)])
def test_close_pair_series_fp32(r, params):
    beta, a, ai, aj = params
    tab = tables()
    got = kernel_close(r, beta, a, ai, aj, tab)
    ref = exact(r, beta, a, ai, aj)
    # B1', B2' are O(1) (relative error at FP32 level); B3' grows like 1/r (relative as well)
    for g, e in zip(got, ref):
        assert abs(g - e) <= 2e-6 * max(abs(e), 1e-3), (r, params, got, ref)


def test_series_tables_match_the_generator():
    """The tables in the kernel are those close_series.py derives (exact rationals)."""
    import importlib.util
    path = os.path.join(os.path.dirname(SRC), "close_series.py")
    spec = importlib.util.spec_from_file_location("close_series", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    gen = mod.tables()
    tab = tables()
    for name, vals in zip(("kD1", "kD2", "kD3", "kPhi3", "kPhi5", "kPsi7"), gen):
        assert np.allclose(tab[name], vals, rtol=1e-15, atol=0)
