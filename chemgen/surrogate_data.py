"""Seeded inputs of the surrogate: training states and initial weights.

Nothing here evaluates a rate or integrates: the labels (the state one flow
step later) come from the GPU integrator, the network arithmetic from the
library.  Recipe of the training states (one mixture, that of
``end_states(mech, default_rng(mix_seed))``, shared with the flame fields the
surrogate serves):

* flame-like states: c ~ U(0, 1), T = 300 + 2200 c + N(0, 50 K) clipped to
  [300, 2500] K, Y = (1 - c) Y_u + c Y_b with each Y_k scaled by a log-normal
  factor exp(0.2 z) and renormalised;
* trajectory starts: T0 ~ U(900, 1500) K with Y = Y_u; the integrator then
  advances them step by step and every visited state is a sample.
"""
from __future__ import annotations

import math
from typing import List, Tuple

import numpy as np

from .fields import P_ATM, end_states
from .mechanism import Mechanism


def flame_like_states(mech: Mechanism, n: int, seed: int, mix_seed: int = 7):
    rng = np.random.default_rng(seed)
    Yu, Yb = end_states(mech, np.random.default_rng(mix_seed))
    c = rng.uniform(0.0, 1.0, size=n)
    T = np.clip(300.0 + 2200.0 * c + rng.normal(0.0, 50.0, size=n), 300.0, 2500.0)
    Y = (1.0 - c)[None, :] * Yu[:, None] + c[None, :] * Yb[:, None]
    Y = Y * np.exp(0.2 * rng.normal(size=Y.shape))
    Y /= Y.sum(axis=0, keepdims=True)
    return T, np.full(n, P_ATM), np.ascontiguousarray(Y)


def trajectory_starts(mech: Mechanism, n: int, seed: int, mix_seed: int = 7):
    rng = np.random.default_rng(seed)
    Yu, _ = end_states(mech, np.random.default_rng(mix_seed))
    T = rng.uniform(900.0, 1500.0, size=n)
    Y = np.repeat(Yu[:, None], n, axis=1)
    return T, np.full(n, P_ATM), np.ascontiguousarray(Y)


def init_params(dims: List[Tuple[int, int]], seed: int) -> np.ndarray:
    """Kaiming-uniform weights (bound sqrt(6 / fan_in) for the GELU layers,
    1 / sqrt(fan_in) for the linear output layer), zero biases, as the flat
    logical vector W1, b1, W2, b2, ... with W of shape (out, in)."""
    rng = np.random.default_rng(seed)
    parts = []
    for i, (fan_in, fan_out) in enumerate(dims):
        bound = math.sqrt(6.0 / fan_in) if i < len(dims) - 1 else 1.0 / math.sqrt(fan_in)
        parts.append(rng.uniform(-bound, bound, size=(fan_out, fan_in)).astype(np.float32).ravel())
        parts.append(np.zeros(fan_out, dtype=np.float32))
    return np.concatenate(parts)


def split_params(flat: np.ndarray, dims: List[Tuple[int, int]]):
    """(W, b) pairs of the flat logical vector, as float64 arrays."""
    out, o = [], 0
    for fan_in, fan_out in dims:
        W = flat[o:o + fan_in * fan_out].reshape(fan_out, fan_in).astype(np.float64)
        o += fan_in * fan_out
        b = flat[o:o + fan_out].astype(np.float64)
        o += fan_out
        out.append((W, b))
    return out


def network_dims(K: int, h1: int = 512, h2: int = 256, h3: int = 128):
    return [(K + 2, h1), (h1, h2), (h2, h3), (h3, K)]


def species_network_dims(K: int, h1: int = 1600, h2: int = 800, h3: int = 400):
    """Layer shapes of one network of the per-species variant (a single output)."""
    return [(K + 2, h1), (h1, h2), (h2, h3), (h3, 1)]


def init_species_params(K: int, h, seed: int) -> np.ndarray:
    """Initial weights of K per-species networks (each as init_params, seeds
    seed, seed + 1, ...), concatenated network by network."""
    dims = species_network_dims(K, *h)
    return np.concatenate([init_params(dims, seed + g) for g in range(K)])


def split_species_params(flat: np.ndarray, K: int, h):
    """The (W, b) lists of the K per-species networks of a flat vector."""
    dims = species_network_dims(K, *h)
    per = sum(a * b + b for a, b in dims)
    return [split_params(flat[g * per:(g + 1) * per], dims) for g in range(K)]


def epoch_orders(n: int, epochs: int, seed: int) -> np.ndarray:
    """A seeded permutation of 0..n-1 per epoch, concatenated (int32)."""
    rng = np.random.default_rng(seed)
    return np.concatenate([rng.permutation(n).astype(np.int32) for _ in range(epochs)])
