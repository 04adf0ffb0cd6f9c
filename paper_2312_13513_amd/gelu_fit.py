"""Coefficients of the branch-free GELU used by the surrogate kernels.

GELU(u) = u Phi(u) with Phi(-|u|) = erfc(z) / 2, z = |u| / sqrt(2).  The
kernels evaluate erfc(z) = t exp(-z^2 + P(t)), t = 1 / (1 + z/2), where P is
a degree-7 polynomial in t.  P is fitted here in FP64 by least squares on
Chebyshev nodes of t in (0, 1] to ln(erfcx(z) / t) (erfcx(z) = exp(z^2)
erfc(z), so the target stays finite for large z).  Run to print the
coefficients and the relative error of an FP32 evaluation of GELU."""
import numpy as np
from scipy.special import erfc, erfcx

DEGREE = 7


def fit(deg: int = DEGREE) -> np.ndarray:
    n = 4000
    k = np.arange(n)
    t = 0.5 * (1.0 + np.cos(np.pi * (k + 0.5) / n))
    y = np.log(erfcx(2.0 * (1.0 / t - 1.0)) / t)
    c = np.polynomial.chebyshev.chebfit(2.0 * t - 1.0, y, deg)
    p_x = np.polynomial.Polynomial(np.polynomial.chebyshev.cheb2poly(c))
    return p_x(np.polynomial.Polynomial([-1.0, 2.0])).coef     # powers of t


def gelu_fp32(u: np.ndarray, coef: np.ndarray) -> np.ndarray:
    f = np.float32
    c = coef.astype(f)
    u = u.astype(f)
    z = (np.abs(u) * f(0.70710678118654752)).astype(f)
    t = (f(1) / (f(1) + f(0.5) * z)).astype(f)
    p = c[-1]
    for ci in c[-2::-1]:
        p = (p * t + ci).astype(f)
    half = (f(0.5) * t * np.exp((p - z * z).astype(f))).astype(f)
    return (u * np.where(u >= 0, f(1) - half, half)).astype(f)


if __name__ == "__main__":
    coef = fit()
    print(", ".join(f"{x:.9e}f" for x in coef))
    u = np.linspace(-20.0, 20.0, 2000001)
    exact = 0.5 * u * erfc(-u / np.sqrt(2.0))
    g = gelu_fp32(u, coef).astype(np.float64)
    m = np.abs(exact) > 1e-37
    print("max relative error of the FP32 GELU:", float((np.abs(g[m] - exact[m]) / np.abs(exact[m])).max()))
