"""Plain numpy oracle of the field-wide thermophysical and transport
properties (paper Section 3.1: the Thermo class computes the thermophysical
and transport properties with Newton's method and temperature polynomials;
Section 2: the molecular transport model is Cantera's).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline may call it; the GPU library never does.

Readings (the paper names the model, not its formulas): Cantera's
mixture-averaged transport.
  * Composition: y_k = max(Y_k, 0) / sum_j max(Y_j, 0); mole fractions
    X_k = (y_k / W_k) / sum_j (y_j / W_j).
  * Pure-species fits, degree-4 polynomials in ln T, lowest power first:
    mu_k = (T^(1/4) P_k(ln T))^2, lam_k = T^(1/2) Q_k(ln T),
    D_jk = T^(3/2) B_jk(ln T) / p (B symmetric in j, k).
  * Viscosity by Wilke's rule: mu = sum_k X_k mu_k / sum_j X_j Phi_kj,
    Phi_kj = (1 + sqrt(mu_k / mu_j) (W_j / W_k)^(1/4))^2 / sqrt(8 (1 + W_k / W_j)).
  * Conductivity by the Mathur-Tondon-Saxena average:
    lam = (sum_k X_k lam_k + 1 / sum_k (X_k / lam_k)) / 2.
  * Mixture-averaged diffusion coefficients:
    D_km = (1 - y_k) / sum_{j != k} X_j / D_jk; for a pure species (the sum
    is zero) D_km = D_kk, the self-diffusion coefficient.
Temperature from mass enthalpy over a field: the oracle's per-cell Newton
(T_from_h) cell by cell, and the mixture cp at the solution.
"""
from __future__ import annotations

import numpy as np

R_U = 8.31446261815324


def poly(c, x):
    """sum_i c[..., i] x^i, lowest power first (Horner)."""
    out = np.zeros(np.broadcast(c[..., 0], x).shape)
    for i in range(c.shape[-1] - 1, -1, -1):
        out = out * x + c[..., i]
    return out


def wilke_phi(mu_k, mu_j, W_k, W_j):
    """Wilke's interaction factor Phi_kj."""
    return (1.0 + np.sqrt(mu_k / mu_j) * (W_j / W_k) ** 0.25) ** 2 / np.sqrt(8.0 * (1.0 + W_k / W_j))


def composition(W, Y):
    """(y, X): clipped and normalised mass fractions and mole fractions, K x n."""
    yp = np.maximum(Y, 0.0)
    y = yp / yp.sum(axis=0)
    c = y / W[:, None]
    return y, c / c.sum(axis=0)


def pure_species(visc, cond, T):
    """(mu_k, lam_k), K x n."""
    lnT = np.log(T)
    mu_k = (T[None, :] ** 0.25 * poly(visc[:, None, :], lnT[None, :])) ** 2
    lam_k = np.sqrt(T)[None, :] * poly(cond[:, None, :], lnT[None, :])
    return mu_k, lam_k


def binary_diffusion(diff, T, p):
    """D_jk, K x K x n."""
    lnT = np.log(T)
    return T ** 1.5 * poly(diff[:, :, None, :], lnT[None, None, :]) / p


def transport(visc, cond, diff, W, T, p, Y):
    """(mu, lam, D): mixture viscosity (Pa s), conductivity (W/(m K)), n each,
    and mixture-averaged diffusion coefficients (m^2/s), K x n."""
    K, n = Y.shape
    y, X = composition(W, Y)
    mu_k, lam_k = pure_species(visc, cond, T)
    mu = np.zeros(n)
    for k in range(K):
        den = np.zeros(n)
        for j in range(K):
            den += X[j] * wilke_phi(mu_k[k], mu_k[j], W[k], W[j])
        mu += X[k] * mu_k[k] / den
    lam = 0.5 * (np.sum(X * lam_k, axis=0) + 1.0 / np.sum(X / lam_k, axis=0))
    Dbin = binary_diffusion(diff, T, p)
    D = np.zeros((K, n))
    for k in range(K):
        s = np.zeros(n)
        for j in range(K):
            if j != k:
                s += X[j] / Dbin[j, k]
        with np.errstate(divide="ignore", invalid="ignore"):
            D[k] = np.where(s > 0.0, (1.0 - y[k]) / s, Dbin[k, k])
    return mu, lam, D


def thermo_field(om, h, Y, T_guess):
    """(T, cp, iters) over a field: T solves h(T, Y) = h by the oracle's
    Newton from T_guess (NaN where it does not converge), cp is the mixture
    cp (J/(kg K)) at that T, iters the Newton iterations (21: no convergence)."""
    n = h.size
    T = np.zeros(n)
    cp = np.zeros(n)
    its = np.zeros(n, dtype=np.int64)
    W = om.W
    for i in range(n):
        T[i], its[i] = om.T_from_h(float(h[i]), Y[:, i], float(T_guess[i]))
        if np.isfinite(T[i]):
            cp_R, _, _ = om.thermo(T[i])
            cp[i] = np.sum(Y[:, i] * cp_R * R_U / W)
        else:
            cp[i] = np.nan
    return T, cp, its
