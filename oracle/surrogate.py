"""Plain FP64 reference of the learned chemistry surrogate (numpy).

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle``): used by the tests to
check the GPU training and inference kernels, never by the library.

What it follows (paper Section 2: the chemistry source is predicted by a DNN
from temperature, pressure and mass fractions, with GELU activations, trained
with Adam; the workload recipe fixes one network: inputs [T, p, BoxCox(Y)],
three hidden layers 512-256-128, outputs the change of the mass fractions over
the flow step):

* encode: x = ([T, p, BC(max(Y,0))] - mu_x) / sigma_x, BC(y) = (y^lam - 1)/lam
  with lam = 0.1; a feature with sigma < 1e-12 maps to 0;
* MLP: h1 = gelu(x W1^T + b1), h2 = gelu(h1 W2^T + b2), h3 = gelu(h2 W3^T + b3),
  out = h3 W4^T + b4, gelu(u) = u (1 + erf(u/sqrt 2)) / 2 (exact form);
* decode: dY = mu_y + sigma_y * out, Y_new = Y + dY;
* loss: mean squared error on the z-scored outputs; Adam with bias correction;
* the per-species variant: one such network per species with a single
  output each, all fed the same input (forward_species, backward_species).

Weights use the (out, in) layout.
"""
from __future__ import annotations

import math
from typing import Dict, List, Tuple

import numpy as np

LAMBDA = 0.1
SIGMA_MIN = 1e-12


def boxcox(y, lam=LAMBDA):
    return (np.power(np.maximum(y, 0.0), lam) - 1.0) / lam


def boxcox_inv(b, lam=LAMBDA):
    return np.power(np.maximum(lam * b + 1.0, 0.0), 1.0 / lam)


def features(T, p, Y):
    """Raw 2 + K features of cells (T (n,), p (n,), Y (K, n)) -> (n, 2+K)."""
    return np.concatenate([T[:, None], p[:, None], boxcox(Y).T], axis=1)


def zscore(raw, mu, sigma):
    out = np.zeros_like(raw)
    ok = sigma >= SIGMA_MIN
    out[:, ok] = (raw[:, ok] - mu[ok]) / sigma[ok]
    return out


def erf(x):
    return np.vectorize(math.erf)(x) if np.ndim(x) else math.erf(x)


def gelu(u):
    return 0.5 * u * (1.0 + erf(u / math.sqrt(2.0)))


def gelu_grad(u):
    return 0.5 * (1.0 + erf(u / math.sqrt(2.0))) + u * np.exp(-0.5 * u * u) / math.sqrt(2.0 * math.pi)


def forward(params: List[Tuple[np.ndarray, np.ndarray]], x):
    """Returns (out, cache) with pre-activations and activations of each layer."""
    acts, pres = [x], []
    h = x
    for li, (W, b) in enumerate(params):
        u = h @ W.T + b
        pres.append(u)
        h = gelu(u) if li < len(params) - 1 else u
        acts.append(h)
    return h, (acts, pres)


def forward_species(nets, x):
    """The paper's per-species variant (Section 2: one network per species,
    each with its own hidden layers and a single output): nets[g] is species
    g's (W, b) list; output column g is its prediction.  Returns (out,
    caches)."""
    outs, caches = [], []
    for params in nets:
        o, c = forward(params, x)
        outs.append(o)
        caches.append(c)
    return np.concatenate(outs, axis=1), caches


def backward_species(nets, caches, out, target):
    """Gradients of mse_loss over all n x G outputs of forward_species: each
    network's own single-output gradient, divided by G (the mean runs over G
    times as many values)."""
    G = len(nets)
    res = []
    for g, params in enumerate(nets):
        gr = backward(params, caches[g], out[:, g:g + 1], target[:, g:g + 1])
        res.append([(gW / G, gb / G) for gW, gb in gr])
    return res


def mse_loss(out, target):
    return float(np.mean((out - target) ** 2))


def backward(params, cache, out, target):
    """Gradients of mse_loss w.r.t. every W and b."""
    acts, pres = cache
    n, m = out.shape
    d = 2.0 * (out - target) / (n * m)
    grads = [None] * len(params)
    for li in range(len(params) - 1, -1, -1):
        W, b = params[li]
        if li < len(params) - 1:
            d = d * gelu_grad(pres[li])
        grads[li] = (d.T @ acts[li], d.sum(axis=0))
        d = d @ W
    return grads


def adam_step(params, grads, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update in place; state = dict(t=int, m=[...], v=[...])."""
    state["t"] += 1
    t = state["t"]
    for i, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
        for j, (P, G) in enumerate(((W, gW), (b, gb))):
            k = 2 * i + j
            state["m"][k] = beta1 * state["m"][k] + (1 - beta1) * G
            state["v"][k] = beta2 * state["v"][k] + (1 - beta2) * G * G
            mhat = state["m"][k] / (1 - beta1 ** t)
            vhat = state["v"][k] / (1 - beta2 ** t)
            P -= lr * mhat / (np.sqrt(vhat) + eps)
    return params


def adam_state(params):
    z = []
    for W, b in params:
        z += [np.zeros_like(W), np.zeros_like(b)]
    return {"t": 0, "m": [a.copy() for a in z], "v": [a.copy() for a in z]}


def cosine_lr(step, total, lr0=1e-3, lr1=1e-5):
    return lr1 + 0.5 * (lr0 - lr1) * (1.0 + math.cos(math.pi * min(step, total) / total))


def predict_cells(params, norm: Dict[str, np.ndarray], T, p, Y):
    """Surrogate prediction of Y_new for cells (before T recovery and checks)."""
    x = zscore(features(T, p, Y), norm["mu_x"], norm["sigma_x"])
    out, _ = forward(params, x)
    dY = norm["mu_y"] + norm["sigma_y"] * out
    return Y + dY.T


# ---------------------------------------------------------------------------
# decode, temperature recovery and acceptance checks (per cell)
# ---------------------------------------------------------------------------

DEFAULT_CHECKS = {
    "elem_tol": 1e-3,      # relative element residual
    "sum_tol": 1e-3,       # |sum Y_new - 1|
    "neg_tol": 1e-6,       # Y_new >= -neg_tol
    "T_out_min": 250.0, "T_out_max": 2600.0,
    "T_in_min": 300.0, "T_in_max": 2500.0,
    "dT_gate": 0.0,        # |T_new - T| <= dT_gate when > 0
}


def apply_cell(om, counts, W, T, Y, yhat, mu_y, sigma_y, checks=None):
    """One cell: returns (ok, T_new, Y_new).  When a check fails the cell keeps
    its input state and ok is False (the caller integrates it instead).

    Order of the steps:
      1. Y1 = Y + mu_y + sigma_y * yhat (the network predicts the z-scored change);
      2. every Y1 finite;
      3. element residual max_e |sum_k n_ke (Y1 - Y)_k / W_k| / max(sum_k n_ke Y_k / W_k, 1e-12);
      4. |sum Y1 - 1|;
      5. min Y1 >= -neg_tol;
      6. Y2 = max(Y1, 0) / sum max(Y1, 0);
      7. T_new from h(T_new, Y2) = h(T, Y) by Newton (the oracle's T_from_h,
         started at T), converged and inside [T_out_min, T_out_max];
      8. input T inside [T_in_min, T_in_max];
      9. optional gate |T_new - T| <= dT_gate."""
    c = dict(DEFAULT_CHECKS)
    if checks:
        c.update(checks)
    Y = np.asarray(Y, dtype=np.float64)
    Y1 = Y + mu_y + sigma_y * np.asarray(yhat, dtype=np.float64)
    fail = (T, Y.copy())
    if not np.all(np.isfinite(Y1)):
        return (False,) + fail
    moles = counts.T / W                          # (E, K): n_ke / W_k
    res = np.abs(moles @ (Y1 - Y))
    ref = np.maximum(moles @ Y, 1e-12)
    if np.max(res / ref) > c["elem_tol"]:
        return (False,) + fail
    if abs(np.sum(Y1) - 1.0) > c["sum_tol"]:
        return (False,) + fail
    if np.min(Y1) < -c["neg_tol"]:
        return (False,) + fail
    Y2 = np.maximum(Y1, 0.0)
    Y2 = Y2 / np.sum(Y2)
    h0 = om.enthalpy(T, Y)
    Tn, _ = om.T_from_h(h0, Y2, T)
    if not np.isfinite(Tn) or Tn < c["T_out_min"] or Tn > c["T_out_max"]:
        return (False,) + fail
    if T < c["T_in_min"] or T > c["T_in_max"]:
        return (False,) + fail
    if c["dT_gate"] > 0.0 and abs(Tn - T) > c["dT_gate"]:
        return (False,) + fail
    return True, Tn, Y2


def to_bf16(x):
    """Round FP32 values to bfloat16 (round to nearest, ties to even); returns
    the rounded values as float64.  NaN stays NaN."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) & 0xFFFF
    r = np.where(np.isnan(f), 0x7FC0, r).astype(np.uint32)
    return (r << 16).view(np.float32).astype(np.float64)


def bf16_bits(x):
    """The 16-bit patterns of to_bf16(x)."""
    return (np.asarray(to_bf16(x), dtype=np.float32).view(np.uint32) >> 16).astype(np.uint16)


def encode_cells(norm, T, p, Y):
    """Network input of cells: z-scored features, FP64 -> FP32 -> BF16."""
    x = zscore(features(T, p, Y), norm["mu_x"], norm["sigma_x"])
    return to_bf16(x.astype(np.float32))


def fit_norm(T, p, Y, Ynext, dt):
    """Normalisation vector: population mean and standard deviation of every
    raw feature and of every dY_k = Ynext_k - Y_k, then dt."""
    raw = features(T, p, Y)
    dY = (np.asarray(Ynext) - np.asarray(Y)).T
    return np.concatenate([raw.mean(axis=0), raw.std(axis=0), dY.mean(axis=0), dY.std(axis=0), [dt]])


def unpack_norm(norm, K):
    nin = K + 2
    return {"mu_x": norm[:nin], "sigma_x": norm[nin:2 * nin], "mu_y": norm[2 * nin:2 * nin + K],
            "sigma_y": norm[2 * nin + K:2 * nin + 2 * K], "dt": float(norm[-1])}
