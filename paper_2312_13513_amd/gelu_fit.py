"""Coefficients of the branch-free GELU used by the surrogate kernels.

GELU(u) = u Phi(u) with Phi(-|u|) = erfc(z) / 2, z = |u| / sqrt(2).  The
form erfc(z) = t exp(-z^2 + P(t)), t = 1 / (1 + z/2), is the one of the
Numerical Recipes routine erfcc (Press et al., Numerical Recipes, section
6.2, after Chebyshev fitting); P, a polynomial in t, is refitted here in FP64
by least squares on Chebyshev nodes of t in (0, 1] to ln(erfcx(z) / t)
(erfcx(z) = exp(z^2) erfc(z), so the target stays finite for large z).

The kernels evaluate it through the hardware base-2 exponential, with the
factor 1/2 of Phi and log2(e) folded into the coefficients:
    Phi(-|u|) = t 2^(Q(t) - u^2 log2(e) / 2),   Q = log2(e) P - 1,
and take the sign with one fused multiply-add:
    GELU(u) = max(u, 0) - |u| Phi(-|u|).
Run to print the coefficients of Q and the relative error of an FP32
evaluation of GELU in that order of operations."""
import numpy as np
from scipy.special import erfc, erfcx

DEGREE = 7
LOG2E = 1.4426950408889634


def fit(deg: int = DEGREE) -> np.ndarray:
    """Coefficients of P (powers of t)."""
    n = 4000
    k = np.arange(n)
    t = 0.5 * (1.0 + np.cos(np.pi * (k + 0.5) / n))
    y = np.log(erfcx(2.0 * (1.0 / t - 1.0)) / t)
    c = np.polynomial.chebyshev.chebfit(2.0 * t - 1.0, y, deg)
    p_x = np.polynomial.Polynomial(np.polynomial.chebyshev.cheb2poly(c))
    return p_x(np.polynomial.Polynomial([-1.0, 2.0])).coef     # powers of t


def kernel_coefficients(deg: int = DEGREE) -> np.ndarray:
    """Coefficients of Q = log2(e) P - 1 (powers of t), as FP32."""
    q = fit(deg) * LOG2E
    q[0] -= 1.0
    return q.astype(np.float32)


def gelu_fp32(u: np.ndarray, q: np.ndarray) -> np.ndarray:
    """GELU in FP32 in the kernels' order of operations."""
    f = np.float32
    u = u.astype(f)
    a = np.abs(u)
    t = (f(1) / (a * f(0.35355339059327373) + f(1))).astype(f)
    p = q[-1]
    for qi in q[-2::-1]:
        p = (p * t + qi).astype(f)
    arg = ((u * u).astype(f) * f(-LOG2E / 2) + p).astype(f)
    half = (t * np.exp2(arg)).astype(f)
    return (-a * half + np.maximum(u, f(0))).astype(f)


if __name__ == "__main__":
    q = kernel_coefficients()
    print(", ".join(f"{x:.9e}f" for x in q))
    u = np.linspace(-20.0, 20.0, 2000001)
    exact = 0.5 * u * erfc(-u / np.sqrt(2.0))
    g = gelu_fp32(u, q).astype(np.float64)
    m = np.abs(exact) > 1e-37
    print("max relative error of the FP32 GELU:", float((np.abs(g[m] - exact[m]) / np.abs(exact[m])).max()))
