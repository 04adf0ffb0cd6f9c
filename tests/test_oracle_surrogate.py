"""Pins of the FP64 surrogate oracle (network, optimiser, encoding, checks)
against library routines, finite differences and closed forms: none of them
re-types the oracle's own formulas."""
import math

import numpy as np
import pytest
import scipy.special
import scipy.stats
import torch

from oracle import surrogate as S


def _net(rng, dims):
    params = []
    for a, b in zip(dims[:-1], dims[1:]):
        params.append((rng.normal(0, 1 / math.sqrt(a), (b, a)), rng.normal(0, 0.1, b)))
    return params


def _torch_net(params):
    layers = []
    for i, (W, b) in enumerate(params):
        lin = torch.nn.Linear(W.shape[1], W.shape[0]).double()
        with torch.no_grad():
            lin.weight.copy_(torch.tensor(W))
            lin.bias.copy_(torch.tensor(b))
        layers.append(lin)
        if i < len(params) - 1:
            layers.append(torch.nn.GELU(approximate="none"))
    return torch.nn.Sequential(*layers)


def test_gelu_is_x_times_normal_cdf():
    x = np.linspace(-8, 8, 1601)
    ref = x * scipy.stats.norm.cdf(x)
    assert np.max(np.abs(S.gelu(x) - ref)) <= 1e-15 * np.max(np.abs(ref)) + 1e-300
    assert S.gelu(0.0) == 0.0
    tg = torch.nn.functional.gelu(torch.tensor(x), approximate="none").numpy()
    assert np.max(np.abs(S.gelu(x) - tg)) < 1e-14


def test_gelu_grad_central_difference():
    x = np.linspace(-6, 6, 241)
    h = 1e-5
    fd = (S.gelu(x + h) - S.gelu(x - h)) / (2 * h)
    assert np.max(np.abs(S.gelu_grad(x) - fd)) < 1e-9


def test_boxcox_library_and_round_trip():
    y = np.logspace(-30, 0, 301)
    assert np.max(np.abs(S.boxcox(y) - scipy.special.boxcox(y, 0.1))) < 1e-13
    back = S.boxcox_inv(S.boxcox(y))
    # inverting amplifies the rounding of lam*b + 1 = y^lam by 1/lam = 10
    assert np.all(np.abs(back - y) / y <= 20 * 2.0 ** -52 / y ** 0.1)
    assert S.boxcox(np.array([0.0]))[0] == -10.0            # (0 - 1) / 0.1
    assert S.boxcox(np.array([-1e-9]))[0] == -10.0          # negatives clip to 0
    # lambda -> 0 limit is the logarithm
    assert abs(S.boxcox(np.array([0.3]), lam=1e-9)[0] - math.log(0.3)) < 1e-8


def test_zscore_degenerate_feature_maps_to_zero():
    raw = np.array([[1.0, 5.0, 2.0], [3.0, 5.0, 4.0]])
    z = S.zscore(raw, np.array([2.0, 5.0, 3.0]), np.array([1.0, 0.0, 1e-13]))
    assert np.array_equal(z[:, 1], [0.0, 0.0]) and np.array_equal(z[:, 2], [0.0, 0.0])
    assert np.array_equal(z[:, 0], [-1.0, 1.0])


def test_forward_matches_torch():
    rng = np.random.default_rng(3)
    params = _net(rng, [7, 16, 12, 8, 5])
    x = rng.normal(size=(11, 7))
    out, _ = S.forward(params, x)
    ref = _torch_net(params)(torch.tensor(x)).detach().numpy()
    assert np.max(np.abs(out - ref)) < 1e-13


def test_backward_matches_finite_differences_and_autograd():
    rng = np.random.default_rng(4)
    params = _net(rng, [5, 9, 7, 6, 4])
    x = rng.normal(size=(6, 5))
    tgt = rng.normal(size=(6, 4))
    out, cache = S.forward(params, x)
    grads = S.backward(params, cache, out, tgt)
    # autograd (library)
    net = _torch_net(params)
    loss = torch.mean((net(torch.tensor(x)) - torch.tensor(tgt)) ** 2)
    loss.backward()
    lins = [m for m in net if isinstance(m, torch.nn.Linear)]
    for (gW, gb), lin in zip(grads, lins):
        assert np.max(np.abs(gW - lin.weight.grad.numpy())) < 1e-14
        assert np.max(np.abs(gb - lin.bias.grad.numpy())) < 1e-14
    # central differences (brute force) on a few entries of every tensor
    h = 1e-6
    for li in range(len(params)):
        for which in (0, 1):
            P = params[li][which]
            G = grads[li][which]
            for idx in list(np.ndindex(P.shape))[:6]:
                old = P[idx]
                P[idx] = old + h
                lp = S.mse_loss(S.forward(params, x)[0], tgt)
                P[idx] = old - h
                lm = S.mse_loss(S.forward(params, x)[0], tgt)
                P[idx] = old
                assert abs((lp - lm) / (2 * h) - G[idx]) < 1e-8


def test_adam_matches_torch_and_first_step_closed_form():
    rng = np.random.default_rng(5)
    params = _net(rng, [4, 6, 3])
    tparams = [torch.tensor(a.copy(), requires_grad=True) for W, b in params for a in (W, b)]
    opt = torch.optim.Adam(tparams, lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    state = S.adam_state(params)
    first = None
    for step in range(5):
        grads = [(rng.normal(size=W.shape), rng.normal(size=b.shape)) for W, b in params]
        before = [W.copy() for W, _ in params]
        S.adam_step(params, grads, state, 1e-3)
        if step == 0:
            first = (before, grads)
        for t, g in zip(tparams, [a for gg in grads for a in gg]):
            t.grad = torch.tensor(g)
        opt.step()
    for (W, b), tW, tb in zip(params, tparams[0::2], tparams[1::2]):
        assert np.max(np.abs(W - tW.detach().numpy())) < 1e-15
        assert np.max(np.abs(b - tb.detach().numpy())) < 1e-15
    # first step: m_hat = g, v_hat = g^2, so the change is -lr g / (|g| + eps)
    p2 = [(w.copy(), np.zeros(3 if i else 6)) for i, w in enumerate(first[0])]
    st = S.adam_state(p2)
    S.adam_step(p2, first[1], st, 1e-3)
    for (W, _), W0, (gW, _) in zip(p2, first[0], first[1]):
        assert np.max(np.abs((W - W0) + 1e-3 * gW / (np.abs(gW) + 1e-8))) < 1e-15


def test_cosine_schedule_end_points():
    assert S.cosine_lr(0, 100) == pytest.approx(1e-3, rel=1e-15)
    assert S.cosine_lr(100, 100) == pytest.approx(1e-5, rel=1e-12)
    assert S.cosine_lr(50, 100) == pytest.approx(0.5 * (1e-3 + 1e-5), rel=1e-12)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(6)
    x = np.concatenate([rng.normal(size=5000).astype(np.float32),
                        (rng.normal(size=2000) * 1e-30).astype(np.float32),
                        np.array([0.0, -0.0, 1.0, 1.00390625, 1.01171875, 65504.0, 3.0e38, 1e-40],
                                 dtype=np.float32)])
    ref = torch.tensor(x).to(torch.bfloat16).to(torch.float64).numpy()
    got = S.to_bf16(x)
    assert np.array_equal(got, ref)
    assert np.array_equal(S.bf16_bits(x), torch.tensor(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16))


@pytest.fixture(scope="module")
def m35(mech_dir):
    from chemgen.mechanism import read_mechanism
    return read_mechanism(str(mech_dir / "M35.mech"))


def _state(m35):
    from chemgen.fields import zones128
    f = zones128(m35, shape=(4, 4, 4))
    i = int(np.argmax(f.zone == 1))
    return float(f.T[i]), f.Y[:, i].copy()


def test_apply_zero_change_keeps_state(om35, m35):
    T, Y = _state(m35)
    K = m35.K
    mu, sg = np.zeros(K), np.ones(K)
    ok, Tn, Yn = S.apply_cell(om35, m35.counts, m35.molar_masses(), T, Y, np.zeros(K), mu, sg)
    assert ok and abs(Tn - T) < 1e-9 and np.max(np.abs(Yn - Y / Y.sum())) < 1e-15


def test_apply_reaction_move_conserves_elements_and_enthalpy(om35, m35):
    """A change along one reaction's stoichiometry conserves every element
    exactly, so it passes; the recovered temperature keeps the mixture
    enthalpy, and an exothermic move heats the cell."""
    T, Y = _state(m35)
    W = m35.molar_masses()
    r = m35.reactions[0]
    nu = np.zeros(m35.K)
    for k, c in r[0]:
        nu[k] -= c
    for k, c in r[1]:
        nu[k] += c
    dY = 1e-4 * nu * W / np.max(np.abs(nu * W))
    Yr = Y.copy()
    Yr[Yr < 2e-4] = 2e-4                        # room for the move in both directions
    Yr /= Yr.sum()
    ok, Tn, Yn = S.apply_cell(om35, m35.counts, W, T, Yr, dY, np.zeros(m35.K), np.ones(m35.K))
    assert ok
    assert abs(om35.enthalpy(Tn, Yn) - om35.enthalpy(T, Yr)) <= 1e-9 * abs(om35.enthalpy(T, Yr)) + 1e-6
    # heat of this move: -sum_k h_k dY_k / cp (first order) has the sign of T_new - T
    _, h_RT, _ = om35.thermo(T)
    dh = float(np.sum(h_RT * 8.31446261815324 * T / W * dY))
    assert np.sign(Tn - T) == -np.sign(dh)


@pytest.mark.parametrize("bad", ["element", "sum", "negative", "nan", "T_in", "gate"])
def test_apply_checks_fail_and_keep_input(om35, m35, bad):
    T, Y = _state(m35)
    W = m35.molar_masses()
    K = m35.K
    dY = np.zeros(K)
    checks = {}
    if bad == "element":
        dY[int(np.argmax(Y))] = -5e-3              # removes atoms
        dY[int(np.argmin(Y))] += 0.0
    elif bad == "sum":
        dY[:] = 2e-3 / K * 1.0
        checks = {"elem_tol": 1e9}
    elif bad == "negative":
        k = int(np.argmin(Y))
        dY[k] = -Y[k] - 1e-5
        checks = {"elem_tol": 1e9, "sum_tol": 1.0}
    elif bad == "nan":
        dY[0] = np.nan
    elif bad == "T_in":
        checks = {"T_in_min": T + 1.0}
    elif bad == "gate":
        r = m35.reactions[0]
        nu = np.zeros(K)
        for k, c in r[0]:
            nu[k] -= c
        for k, c in r[1]:
            nu[k] += c
        dY = 1e-3 * nu * W / np.max(np.abs(nu * W))
        Y = np.maximum(Y, 2e-3)
        Y /= Y.sum()
        checks = {"dT_gate": 1e-6}
    ok, Tn, Yn = S.apply_cell(om35, m35.counts, W, T, Y, dY, np.zeros(K), np.ones(K), checks)
    assert not ok and Tn == T and np.array_equal(Yn, Y)


def _species_nets(rng, nin, h, G):
    return [_net(rng, [nin, *h, 1]) for _ in range(G)]


def test_species_networks_are_one_block_diagonal_network():
    """G single-output networks on a shared input equal one dense network
    whose first layer stacks their first layers and whose later layers are
    block diagonal (each species' block, zeros between): a structural pin of
    forward_species and backward_species through the single-network oracle,
    itself pinned against torch above."""
    rng = np.random.default_rng(71)
    nin, h, G, n = 7, (5, 4, 3), 4, 11
    nets = _species_nets(rng, nin, h, G)
    dense = []
    for li in range(4):
        Ws = [net[li][0] for net in nets]
        bs = [net[li][1] for net in nets]
        if li == 0:
            W = np.vstack(Ws)
        else:
            W = np.zeros((sum(w.shape[0] for w in Ws), sum(w.shape[1] for w in Ws)))
            r = c = 0
            for w in Ws:
                W[r:r + w.shape[0], c:c + w.shape[1]] = w
                r += w.shape[0]
                c += w.shape[1]
        dense.append((W, np.concatenate(bs)))
    x = rng.normal(0, 1, (n, nin))
    tgt = rng.normal(0, 1, (n, G))
    out_s, caches = S.forward_species(nets, x)
    out_d, cache_d = S.forward(dense, x)
    assert np.allclose(out_s, out_d, rtol=1e-13, atol=1e-14)
    gs = S.backward_species(nets, caches, out_s, tgt)
    gd = S.backward(dense, cache_d, out_d, tgt)
    for g in range(G):
        # the dense gradient's diagonal blocks are the species networks' gradients
        r0 = [g * hh for hh in (*h, 1)]
        c0 = [0] + [g * hh for hh in h]
        for li, size_o in enumerate((*h, 1)):
            size_i = nin if li == 0 else h[li - 1]
            blk = gd[li][0][r0[li]:r0[li] + size_o, c0[li]:c0[li] + size_i]
            assert np.allclose(gs[g][li][0], blk, rtol=1e-12, atol=1e-15)
            assert np.allclose(gs[g][li][1], gd[li][1][r0[li]:r0[li] + size_o], rtol=1e-12, atol=1e-15)


def test_species_backward_finite_differences():
    """Central differences of the mean squared error over all n x G outputs
    against backward_species, on weights and biases of every layer of two of
    the networks (the 1/G factor of the mean included)."""
    rng = np.random.default_rng(72)
    nin, h, G, n = 5, (4, 3, 3), 3, 6
    nets = _species_nets(rng, nin, h, G)
    x = rng.normal(0, 1, (n, nin))
    tgt = rng.normal(0, 1, (n, G))
    out, caches = S.forward_species(nets, x)
    grads = S.backward_species(nets, caches, out, tgt)

    def loss():
        return S.mse_loss(S.forward_species(nets, x)[0], tgt)

    eps = 1e-6
    for g in (0, 2):
        for li in range(4):
            for which in (0, 1):
                P = nets[g][li][which]
                idx = tuple(rng.integers(0, d) for d in P.shape)
                keep = P[idx]
                P[idx] = keep + eps
                lp = loss()
                P[idx] = keep - eps
                lm = loss()
                P[idx] = keep
                fd = (lp - lm) / (2 * eps)
                an = grads[g][li][which][idx]
                assert abs(fd - an) <= 1e-7 + 1e-5 * abs(fd), (g, li, which, fd, an)
