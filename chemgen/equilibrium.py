"""Ideal-gas chemical equilibrium at fixed (T, p) for building input fields.

Used only to construct the unburnt and burnt compositions of the synthetic
flame fields (cells at c = 0 or c = 1 then start at equilibrium).  It carries
its own NASA-7 Gibbs evaluation; it is never called by the integrators.

Method: element potentials.  At equilibrium the mole fractions are
``X_k = (p0/p) exp(-g_k + n_k . lam)`` with g_k = G_k/(R T).  For a trial total
mole number N the potentials lam minimise the convex function
``Phi(lam) = N sum_k X_k(lam) - b . lam`` (its gradient is the element balance);
N itself is then fixed by ``sum_k X_k = 1`` with bisection in log N, which is
monotone because every species carries at least one atom.
"""
from __future__ import annotations

import math

import numpy as np

P_STD = 101325.0


def nasa_coeff_rows(nasa: np.ndarray, T: float) -> np.ndarray:
    lo = nasa[:, 3:10]
    hi = nasa[:, 10:17]
    use_lo = (T < nasa[:, 1])[:, None]
    return np.where(use_lo, lo, hi)


def gibbs_over_RT(nasa: np.ndarray, T: float) -> np.ndarray:
    a = nasa_coeff_rows(nasa, T)
    h = a[:, 0] + a[:, 1] * T / 2 + a[:, 2] * T ** 2 / 3 + a[:, 3] * T ** 3 / 4 + a[:, 4] * T ** 4 / 5 + a[:, 5] / T
    s = (a[:, 0] * math.log(T) + a[:, 1] * T + a[:, 2] * T ** 2 / 2 + a[:, 3] * T ** 3 / 3
         + a[:, 4] * T ** 4 / 4 + a[:, 6])
    return h - s


def _minimise_dual(g, n, b, N, lam):
    for _ in range(500):
        u = -g + n @ lam
        X = np.exp(u)
        grad = N * (n.T @ X) - b
        H = N * (n.T * X) @ n
        try:
            step = np.linalg.solve(H, -grad)
        except np.linalg.LinAlgError:
            step = -grad
        big = np.max(np.abs(step))
        if not np.isfinite(big):
            step = -grad / max(np.max(np.abs(grad)), 1e-300)
            big = np.max(np.abs(step))
        if big > 5.0:
            step = step * (5.0 / big)
        phi0 = N * X.sum() - b @ lam
        slope = grad @ step
        t = 1.0
        while True:
            lam_new = lam + t * step
            u2 = -g + n @ lam_new
            if np.all(u2 < 700.0):
                phi = N * np.exp(u2).sum() - b @ lam_new
                if phi <= phi0 + 1e-4 * t * slope or t < 1e-6:
                    break
            t *= 0.5
            if t < 1e-20:
                break
        lam = lam_new
        if np.max(np.abs(t * step)) <= 1e-15 * (1.0 + np.max(np.abs(lam))):
            break
    return lam


def equilibrium_mass_fractions(mech, T: float, p: float, b: np.ndarray) -> np.ndarray:
    """Equilibrium mass fractions for element moles ``b`` (mol of atoms per kg)."""
    n = mech.counts.astype(np.float64)
    W = mech.molar_masses()
    g = gibbs_over_RT(mech.nasa, T) + math.log(p / P_STD)
    atoms = n.sum(axis=1)
    sb = b.sum()
    lo, hi = math.log(sb / atoms.max()) - 1e-9, math.log(sb / atoms.min()) + 1e-9
    # start with all potentials equal and the most stable species at X = 1
    lam = np.full(n.shape[1], np.min(g / atoms))
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        lam = _minimise_dual(g, n, b, math.exp(mid), lam)
        s = np.exp(-g + n @ lam).sum()
        if s > 1.0:
            lo = mid
        else:
            hi = mid
        if hi - lo < 1e-15:
            break
    N = math.exp(0.5 * (lo + hi))
    lam = _minimise_dual(g, n, b, N, lam)
    X = np.exp(-g + n @ lam)
    Nk = N * X
    Y = Nk * W
    return Y / Y.sum()


def element_moles(mech, Y: np.ndarray) -> np.ndarray:
    """Moles of each element per kg of mixture for mass fractions Y (K,)."""
    return mech.counts.T.astype(np.float64) @ (Y / mech.molar_masses())
