"""Seeded species transport data (input building only).

The paper computes transport properties on the GPU beside the chemistry
(Sections 3.1 and 3.2: the Thermo class, compute-bound property kernels).
Its mechanisms' transport files are not available, so every species gets
synthetic Lennard-Jones parameters (collision diameter sigma, well depth
eps/k) drawn from a seed, from which pure-species viscosity, conductivity and
binary diffusion coefficients are evaluated on a temperature grid by
kinetic-theory formulas (Chapman-Enskog with the Neufeld-Janzen-Aziz 1972
collision-integral correlations, a modified Eucken factor for conductivity)
and fitted, per species and per pair, by polynomials of degree 4 in ln T in
the forms of Cantera's mixture-averaged model:

    viscosity     mu_k   = (T^(1/4) P_k(ln T))^2
    conductivity  lam_k  = T^(1/2) Q_k(ln T)
    diffusion     D_jk   = T^(3/2) B_jk(ln T) / p        (B symmetric)

The fitted coefficients are the inputs of the property kernels; the mixture
rules that combine them belong to the method (the oracle and the GPU
library each implement them).
"""
from __future__ import annotations

import math

import numpy as np

from .mechanism import R_U

T_FIT = np.linspace(300.0, 3500.0, 65)
AVOGADRO = 6.02214076e23
KB = 1.380649e-23


def _omega22(ts):
    return 1.16145 * ts ** -0.14874 + 0.52487 * np.exp(-0.77320 * ts) + 2.16178 * np.exp(-2.43787 * ts)


def _omega11(ts):
    return (1.06036 * ts ** -0.15610 + 0.19300 * np.exp(-0.47635 * ts) + 1.03587 * np.exp(-1.52996 * ts)
            + 1.76474 * np.exp(-3.89411 * ts))


def lennard_jones(mech, seed: int):
    """Seeded (sigma in m, eps/k in K) per species, growing with atom count."""
    rng = np.random.default_rng(seed)
    atoms = mech.counts.sum(axis=1)
    sigma = (2.5 + 0.4 * (atoms - 1) + rng.uniform(0.0, 0.6, mech.K)) * 1e-10
    eps = 60.0 + 90.0 * (atoms - 1) + rng.uniform(0.0, 120.0, mech.K)
    return sigma, eps


def _mu_kinetic(W, sigma, eps, T):
    m = W / AVOGADRO
    return 5.0 / 16.0 * np.sqrt(math.pi * m * KB * T) / (math.pi * sigma ** 2 * _omega22(T / eps))


def kinetic_viscosity(mech, seed: int, T=T_FIT):
    """Chapman-Enskog viscosity of every species (K x len(T)), Pa s."""
    sigma, eps = lennard_jones(mech, seed)
    W = mech.molar_masses()
    return np.array([_mu_kinetic(W[k], sigma[k], eps[k], T) for k in range(mech.K)])


def transport_fits(mech, seed: int):
    """(visc K x 5, cond K x 5, diff K x K x 5) coefficients, lowest power first."""
    K = mech.K
    W = mech.molar_masses()                                   # kg/mol
    atoms = mech.counts.sum(axis=1)
    sigma, eps = lennard_jones(mech, seed)
    m = W / AVOGADRO
    lnT = np.log(T_FIT)
    visc = np.zeros((K, 5))
    cond = np.zeros((K, 5))
    for k in range(K):
        mu = _mu_kinetic(W[k], sigma[k], eps[k], T_FIT)
        # monatomic-like part plus an internal-energy part (modified Eucken)
        cv_int = 1.5 * (atoms[k] > 1) + 0.5 * (atoms[k] > 2)
        lam = mu / W[k] * R_U * (15.0 / 4.0 + 1.32 * cv_int)
        visc[k] = np.polyfit(lnT, np.sqrt(mu) / T_FIT ** 0.25, 4)[::-1]
        cond[k] = np.polyfit(lnT, lam / np.sqrt(T_FIT), 4)[::-1]
    diff = np.zeros((K, K, 5))
    for j in range(K):
        for k in range(j, K):
            s = 0.5 * (sigma[j] + sigma[k])
            e = math.sqrt(eps[j] * eps[k])
            mjk = m[j] * m[k] / (m[j] + m[k])
            ts = T_FIT / e
            # D p in Pa m^2/s
            Dp = 3.0 / 16.0 * np.sqrt(2.0 * math.pi * (KB * T_FIT) ** 3 / mjk) / (math.pi * s ** 2 * _omega11(ts))
            c = np.polyfit(lnT, Dp / T_FIT ** 1.5, 4)[::-1]
            diff[j, k] = c
            diff[k, j] = c
    return visc, cond, diff
