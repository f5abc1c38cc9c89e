"""Coefficients of the short-range series used by the FP32 pair kernels for very close pairs.

For r -> 0 the Ewald radial functions B_n ~ (2n-1)!!/r^(2n+1) and the Thole terms cancel to
O(1) values, which FP32 cannot resolve when each term is computed separately.  With x = beta r
and eps = A r^3 (A = a / sqrt(alpha_i alpha_j)) the damped functions are rewritten as sums of
well-conditioned pieces:

    B_n - (2n-1)!!/r^(2n+1) = beta^(2n+1) d_n(x^2)            (power series in x^2)
    B1' = beta^3 d_1 + A phi3(eps),              phi3 = lambda3 / eps
    B2' = beta^5 d_2 + 3 A^2 r phi5(eps),        phi5 = lambda5 / eps^2
    B3' = beta^7 d_3 + 15 A^2 psi7(eps) / r,     psi7 = lambda7 / eps^2

with lambda3 = 1 - e^-eps, lambda5 = 1 - (1+eps) e^-eps, lambda7 = 1 - (1+eps+3/5 eps^2) e^-eps.
The d_n follow from B_0 = erfc(x)/r and B_n = ((2n-1) B_(n-1) + 2^n beta^(2n-1) e^(-x^2)/sqrt(pi)) / r^2:
d_0 = -erf(x)/x and d_n = ((2n-1) d_(n-1) + 2^n e^(-x^2)/sqrt(pi)) / x^2, where the constant terms cancel.

Run to print the coefficient tables (exact rationals, then as floats) used in realspace.hip.
"""
from fractions import Fraction
from math import factorial, pi, sqrt

NX = 9     # terms in x^2
NE = 12    # terms in eps


def d_series(n_max=3, terms=NX + 4):
    """Coefficients of d_n(x^2) (in units of 1/sqrt(pi)): d_n = (1/sqrt(pi)) sum_k c[n][k] x^(2k)."""
    # d_0 = -erf(x)/x = -(2/sqrt(pi)) sum_k (-1)^k x^(2k) / (k! (2k+1))
    c = [[Fraction(-2 * (-1) ** k, factorial(k) * (2 * k + 1)) for k in range(terms)]]
    # e^(-x^2) = sum_k (-1)^k x^(2k) / k!
    g = [Fraction((-1) ** k, factorial(k)) for k in range(terms)]
    for n in range(1, n_max + 1):
        num = [(2 * n - 1) * c[n - 1][k] + 2 ** n * g[k] for k in range(terms)]
        assert num[0] == 0, (n, num[0])
        c.append(num[1:] + [Fraction(0)])
    return c


def phi_series(terms=NE):
    """phi3 = (1 - e^-e)/e, phi5 = (1 - (1+e) e^-e)/e^2, psi7 = (1 - (1+e+3/5 e^2) e^-e)/e^2."""
    ex = [Fraction((-1) ** k, factorial(k)) for k in range(terms + 4)]   # e^-e
    lam3 = [-ex[k] for k in range(terms + 4)]
    lam3[0] += 1
    lam5 = [-(ex[k] + (ex[k - 1] if k >= 1 else 0)) for k in range(terms + 4)]
    lam5[0] += 1
    lam7 = [-(ex[k] + (ex[k - 1] if k >= 1 else 0) + (Fraction(3, 5) * ex[k - 2] if k >= 2 else 0))
            for k in range(terms + 4)]
    lam7[0] += 1
    assert lam3[0] == 0 and lam5[0] == 0 and lam5[1] == 0 and lam7[0] == 0 and lam7[1] == 0
    return lam3[1:terms + 1], lam5[2:terms + 2], lam7[2:terms + 2]


def tables():
    c = d_series()
    p3, p5, p7 = phi_series()
    s = 1.0 / sqrt(pi)
    return ([float(v) * s for v in c[1][:NX]], [float(v) * s for v in c[2][:NX]], [float(v) * s for v in c[3][:NX]],
            [float(v) for v in p3], [float(v) for v in p5], [float(v) for v in p7])


if __name__ == "__main__":
    names = ("kD1", "kD2", "kD3", "kPhi3", "kPhi5", "kPsi7")
    for name, vals in zip(names, tables()):
        body = ",\n    ".join(", ".join(f"{v:.17e}" for v in vals[i:i + 3]) for i in range(0, len(vals), 3))
        print(f"constexpr double {name}[{len(vals)}] = {{\n    {body}}};")
