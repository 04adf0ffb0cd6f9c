"""Seeded synthetic cell states (T, p, Y) shaped like the paper's workloads.

Each workload is a batch of CFD cells advanced over one flow step dt:

* ``cells4096``   - 4,096 cells of the 9-species mechanism, T uniform in
  [900, 2200] K, Y from Dirichlet(1), dt = 1e-6 s (small parity case).
* ``flame64``     - 64^3 = 262,144 cells of the 9-species mechanism on a smooth
  progress-variable field (Table 1's middle mesh), dt = 1e-6 s.
* ``zones128``    - 128^3 cells of the 35-species mechanism: 60 % cold, 10 %
  thin flame front, 30 % burnt (uneven stiffness), dt = 1e-5 s.
* ``flame256x128x128`` / ``flame256`` - 35-species flame fields of 4.2M and
  16.8M cells (the TGV mesh of Section 4.1 is 256^3), dt = 1e-5 s.
* ``tgv_share``   - 256 x 128 x 128 = 4,194,304 cells of the 9-species
  mechanism: one GPU's quarter of the 256^3 TGV mesh run on four GPUs
  (Section 4.1), a smooth flame field; the workload of the property
  kernels, with ``newton_guess`` standing in for the previous step's T.

Arrays use the structure-of-arrays layout of the library: ``Y`` has shape
(K, n), one contiguous row per species.  Nothing here evaluates a rate.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Tuple

import numpy as np

from .equilibrium import element_moles, equilibrium_mass_fractions
from .mechanism import Mechanism, standard_mechanism

P_ATM = 101325.0


@dataclasses.dataclass
class Field:
    name: str
    mech_name: str
    T: np.ndarray          # (n,) K
    p: np.ndarray          # (n,) Pa
    Y: np.ndarray          # (K, n) mass fractions
    dt: float
    rtol: float = 1e-8
    atol: float = 1e-12
    c: Optional[np.ndarray] = None   # progress variable, when the field has one
    zone: Optional[np.ndarray] = None

    @property
    def n(self) -> int:
        return self.T.shape[0]


def c_field(shape: Tuple[int, int, int], rng: np.random.Generator, nmodes: int = 8) -> np.ndarray:
    """Progress variable in [0, 1]: min-max normalised sum of ``nmodes`` periodic
    Fourier modes a_m cos(2 pi k_m . x + phi_m) with integer wave vectors
    k_m in {-3..3}^3 minus the origin, a_m ~ U[0.5, 1], phi_m ~ U[0, 2 pi)."""
    kv = np.array([(i, j, k) for i in range(-3, 4) for j in range(-3, 4) for k in range(-3, 4)
                   if (i, j, k) != (0, 0, 0)], dtype=np.float64)
    sel = rng.integers(0, len(kv), size=nmodes)
    amp = rng.uniform(0.5, 1.0, size=nmodes)
    phi = rng.uniform(0.0, 2.0 * math.pi, size=nmodes)
    axes = [np.arange(s, dtype=np.float64) / s for s in shape]
    s = np.zeros(shape, dtype=np.float64)
    for m in range(nmodes):
        k = kv[sel[m]]
        ph = (2.0 * math.pi * (k[0] * axes[0][:, None, None] + k[1] * axes[1][None, :, None]
                               + k[2] * axes[2][None, None, :]) + phi[m])
        s += amp[m] * np.cos(ph)
    s = s.reshape(-1)
    return (s - s.min()) / (s.max() - s.min())


def end_states(mech: Mechanism, rng: np.random.Generator, T_u=300.0, T_b=2200.0, p=P_ATM):
    """Unburnt and burnt compositions: equilibria at T_u and T_b for one element
    composition taken from a Dirichlet(1) draw of species mass fractions."""
    Y0 = rng.dirichlet(np.ones(mech.K))
    b = element_moles(mech, Y0)
    Yu = equilibrium_mass_fractions(mech, T_u, p, b)
    Yb = equilibrium_mass_fractions(mech, T_b, p, b)
    return Yu, Yb


def cells4096(mech: Optional[Mechanism] = None, n: int = 4096, seed: int = 101) -> Field:
    mech = mech or standard_mechanism("M9")
    rng = np.random.default_rng(seed)
    T = rng.uniform(900.0, 2200.0, size=n)
    Y = rng.dirichlet(np.ones(mech.K), size=n).T.copy()
    return Field("cells4096", "M9", T, np.full(n, P_ATM), Y, 1e-6)


def flame_field(mech: Mechanism, shape, seed: int, dt: float, name: str, mech_name: str,
                mix_seed: Optional[int] = None) -> Field:
    """Smooth flame field.  The unburnt/burnt end states come from the field's
    own random stream, or from ``default_rng(mix_seed)`` when given (the same
    mixture as the surrogate's training data of that seed)."""
    rng = np.random.default_rng(seed)
    c = c_field(shape, rng)
    Yu, Yb = end_states(mech, rng if mix_seed is None else np.random.default_rng(mix_seed))
    T = 300.0 + 1900.0 * c
    Y = (1.0 - c)[None, :] * Yu[:, None] + c[None, :] * Yb[:, None]
    return Field(name, mech_name, T, np.full(c.size, P_ATM), Y, dt, c=c)


def flame64(mech: Optional[Mechanism] = None, seed: int = 102) -> Field:
    return flame_field(mech or standard_mechanism("M9"), (64, 64, 64), seed, 1e-6, "flame64", "M9")


def zones128(mech: Optional[Mechanism] = None, seed: int = 103, shape=(128, 128, 128),
             shuffle: bool = False) -> Field:
    """Three stiffness zones split by quantiles of a smooth c-field: lowest 60 %
    cold (T ~ U[300, 600], Y = unburnt), next 10 % flame front (T ~ U[1200, 2000],
    Y mixed at c' = (T - 300)/1900), top 30 % burnt (T ~ U[2000, 2200], Y = burnt)."""
    mech = mech or standard_mechanism("M35")
    rng = np.random.default_rng(seed)
    c = c_field(shape, rng)
    Yu, Yb = end_states(mech, rng)
    n = c.size
    order = np.argsort(c, kind="stable")
    rank = np.empty(n, dtype=np.int64)
    rank[order] = np.arange(n)
    zone = np.where(rank < int(0.6 * n), 0, np.where(rank < int(0.7 * n), 1, 2))
    T = np.empty(n)
    T[zone == 0] = rng.uniform(300.0, 600.0, size=int((zone == 0).sum()))
    T[zone == 1] = rng.uniform(1200.0, 2000.0, size=int((zone == 1).sum()))
    T[zone == 2] = rng.uniform(2000.0, 2200.0, size=int((zone == 2).sum()))
    cm = np.where(zone == 0, 0.0, np.where(zone == 2, 1.0, (T - 300.0) / 1900.0))
    Y = (1.0 - cm)[None, :] * Yu[:, None] + cm[None, :] * Yb[:, None]
    if shuffle:
        perm = rng.permutation(n)
        T, Y, zone, c = T[perm], Y[:, perm], zone[perm], c[perm]
    return Field("zones128" + ("_shuffled" if shuffle else ""), "M35", T, np.full(n, P_ATM),
                 np.ascontiguousarray(Y), 1e-5, c=c, zone=zone)


def flame256x128x128(mech: Optional[Mechanism] = None, seed: int = 104) -> Field:
    return flame_field(mech or standard_mechanism("M35"), (256, 128, 128), seed, 1e-5,
                       "flame256x128x128", "M35", mix_seed=7)


def flame256(mech: Optional[Mechanism] = None, seed: int = 105) -> Field:
    return flame_field(mech or standard_mechanism("M35"), (256, 256, 256), seed, 1e-5, "flame256", "M35",
                       mix_seed=7)


def tgv_share(mech: Optional[Mechanism] = None, seed: int = 106) -> Field:
    return flame_field(mech or standard_mechanism("M9"), (256, 128, 128), seed, 1e-6, "tgv_share", "M9")


def newton_guess(T: np.ndarray, seed: int, spread: float = 20.0) -> np.ndarray:
    """T plus a seeded uniform offset in [-spread, spread] K: the previous
    flow step's temperature as the start of the enthalpy Newton."""
    return T + np.random.default_rng(seed).uniform(-spread, spread, T.shape[0])


def subset(field: Field, idx: np.ndarray, name_suffix: str = "_sub") -> Field:
    return dataclasses.replace(field, name=field.name + name_suffix, T=field.T[idx].copy(),
                               p=field.p[idx].copy(), Y=np.ascontiguousarray(field.Y[:, idx]),
                               c=None if field.c is None else field.c[idx],
                               zone=None if field.zone is None else field.zone[idx])


def seeded_sample(n_total: int, n_sample: int, seed: int = 7) -> np.ndarray:
    """A seeded uniform sample of cell indices, sorted."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n_total, size=min(n_sample, n_total), replace=False))
