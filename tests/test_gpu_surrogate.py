"""GPU parity of the learned surrogate (called through the C ABI) against the
FP64 oracle: input encoding, BF16 MFMA forward pass, gradients, Adam, the
decode/check step, fallback to the integrator, training and the weights file.

Tolerances for the BF16 network come from its arithmetic: weights and inputs
are the same BF16 values on both sides; the GPU rounds every hidden
activation to BF16 (unit roundoff 2^-8) and accumulates in FP32, so per layer
|du| <= |W| |dh| + K 2^-24 |W| |h| and |dh'| <= 1.13 |du| + 2^-8 |gelu(u)|,
propagated from the oracle's own |W| and |h| (a first-order bound, taken
with a factor 2)."""
import os
import sys

import numpy as np
import pytest

from test_gpu_integrate import _say

pytestmark = pytest.mark.gpu

U_BF16 = 2.0 ** -8
GELU_LIP = 1.13


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


@pytest.fixture(scope="module")
def mechs(mech_dir, torch):
    from paper_2312_13513_amd import chem
    m9 = chem.Mechanism(str(mech_dir / "M9.mech"), 0)
    m35 = chem.Mechanism(str(mech_dir / "M35.mech"), 0)
    yield {"M9": m9, "M35": m35}
    m9.close()
    m35.close()


@pytest.fixture(scope="module")
def m35py(mech_dir):
    from chemgen.mechanism import read_mechanism
    return read_mechanism(str(mech_dir / "M35.mech"))


def _dev(torch, a, dtype=None):
    import torch as t
    return t.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda:0")


def _synthetic_norm(T, p, Y, K, rng, dy_scale=1e-4):
    """A normalisation vector from the states themselves (test input, not an
    output of either side); dY statistics are synthetic."""
    from oracle import surrogate as S
    raw = S.features(T, p, Y)
    mu_y = rng.normal(0.0, 0.1, K) * dy_scale
    sig_y = rng.uniform(0.5, 1.5, K) * dy_scale
    return np.concatenate([raw.mean(axis=0), raw.std(axis=0), mu_y, sig_y, [1e-5]])


def _surr(chem, mech, K, h=(512, 256, 128), seed=11):
    from chemgen.surrogate_data import init_params, network_dims
    s = chem.Surrogate(mech, *h)
    dims = network_dims(K, *h)
    flat = init_params(dims, seed)
    # non-zero biases exercise the bias epilogues
    rng = np.random.default_rng(seed + 1)
    o = 0
    for fi, fo in dims:
        o += fi * fo
        flat[o:o + fo] = rng.normal(0, 0.05, fo).astype(np.float32)
        o += fo
    s.set_params(flat)
    return s, dims, flat


def test_encode_bit_exact(torch, mechs, m35py):
    from chemgen.fields import zones128
    from oracle import surrogate as S
    from paper_2312_13513_amd import chem
    f = zones128(m35py, shape=(16, 16, 16))
    K = m35py.K
    rng = np.random.default_rng(1)
    norm = _synthetic_norm(f.T, f.p, f.Y, K, rng)
    s = chem.Surrogate(mechs["M35"], 64, 64, 64)
    s.set_norm(norm)
    X = torch.zeros((f.n, 64), dtype=torch.int16, device="cuda:0")
    s.encode(_dev(torch, f.T), _dev(torch, f.p), _dev(torch, f.Y), X)
    torch.cuda.synchronize()
    got = X.cpu().numpy().view(np.uint16)
    ref = np.zeros_like(got)
    ref[:, :K + 2] = S.bf16_bits(S.encode_cells(S.unpack_norm(norm, K), f.T, f.p, f.Y))
    diff = got != ref
    _say(f"[encode] {diff.sum()} of {diff.size} BF16 codes differ")
    # both sides decide the code in FP64 -> FP32 -> BF16; only a 1-ulp pow
    # difference landing on a rounding boundary can flip one
    assert diff.sum() <= max(1, diff.size // 100000)
    if diff.any():
        assert np.all(np.abs(got[diff].astype(np.int32) - ref[diff].astype(np.int32)) == 1)
    s.close()


def _forward_bound(params_bf, x):
    """Oracle forward plus the elementwise bound of the GPU's deviation."""
    from oracle import surrogate as S
    h, e = x, np.zeros_like(x)
    for li, (W, b) in enumerate(params_bf):
        aW = np.abs(W)
        u = h @ W.T + b
        eu = e @ aW.T + W.shape[1] * 2.0 ** -24 * (np.abs(h) @ aW.T + np.abs(b))
        if li < len(params_bf) - 1:
            g = S.gelu(u)
            e = GELU_LIP * eu + U_BF16 * np.abs(g)
            h = g
        else:
            return u, eu


@pytest.mark.parametrize("rows,path", [(1, 1), (63, 1), (2050, 1), (1, 2), (63, 2), (2050, 2)])
def test_forward_parity(torch, mechs, rows, path):
    """path 1: one GEMM per layer; path 2: the fused kernel."""
    from chemgen.surrogate_data import split_params
    from oracle import surrogate as S
    from paper_2312_13513_amd import chem
    K = 35
    s, dims, flat = _surr(chem, mechs["M35"], K)
    rng = np.random.default_rng(rows)
    x = S.to_bf16(rng.normal(0, 1, (rows, K + 2)).astype(np.float32))
    Xb = np.zeros((rows, 64), dtype=np.uint16)
    Xb[:, :K + 2] = S.bf16_bits(x)
    X = torch.tensor(Xb.view(np.int16), device="cuda:0")
    out = torch.zeros((rows, s.nout_pad), dtype=torch.float32, device="cuda:0")
    s.forward(X, out, path=path)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    params_bf = [(S.to_bf16(W.astype(np.float32)), b) for W, b in split_params(flat, dims)]
    ref, bound = _forward_bound(params_bf, x)
    err = np.abs(got[:, :K] - ref)
    rel = np.linalg.norm(got[:, :K] - ref) / np.linalg.norm(ref)
    _say(f"[forward rows={rows}] max err {err.max():.3e}, max err/bound {(err / (2 * bound + 1e-30)).max():.3f}, "
         f"rel-L2 {rel:.3e}")
    assert np.all(err <= 2.0 * bound + 1e-6)
    assert np.all(got[:, K:] == 0.0)          # padded outputs: zero rows of W4, zero bias
    assert rel < 1e-2
    s.close()


@pytest.mark.parametrize("h", [(512, 256, 128), (64, 64, 64), (128, 512, 64)])
def test_fused_forward_bitwise_layered(torch, mechs, h):
    """The fused kernel against the layer-by-layer GEMMs: the same MFMA
    accumulation order and epilogues, so the outputs are equal bit for bit;
    row counts that leave a partial 64-row tile, several tiles, and one
    larger than the GEMM path's 262,144-row chunk."""
    from oracle import surrogate as S
    from paper_2312_13513_amd import chem
    K = 35
    s, dims, flat = _surr(chem, mechs["M35"], K, h=h)
    for rows in (1, 65, 4097, 300000):
        rng = np.random.default_rng(rows)
        x = S.to_bf16(rng.normal(0, 1, (rows, K + 2)).astype(np.float32))
        Xb = np.zeros((rows, 64), dtype=np.uint16)
        Xb[:, :K + 2] = S.bf16_bits(x)
        X = torch.tensor(Xb.view(np.int16), device="cuda:0")
        o1 = torch.full((rows, s.nout_pad + 3), -9.0, dtype=torch.float32, device="cuda:0")
        o2 = torch.full((rows, s.nout_pad + 3), -9.0, dtype=torch.float32, device="cuda:0")
        s.forward(X, o1, path=1)
        s.forward(X, o2, path=2)
        torch.cuda.synchronize()
        assert torch.equal(o1, o2), f"rows {rows}: fused and layered outputs differ"
        assert torch.all(o2[:, s.nout_pad:] == -9.0)          # columns past the outputs untouched
    _say(f"[fused forward {h}] equal to the layered GEMMs bit for bit at 1, 65, 4097 and 300000 rows")
    s.close()


def test_fused_forward_rejects_wide_layers(torch, mechs):
    from paper_2312_13513_amd import chem
    s, dims, flat = _surr(chem, mechs["M9"], 9, h=(1024, 64, 64))
    X = torch.zeros((4, 64), dtype=torch.int16, device="cuda:0")
    out = torch.zeros((4, s.nout_pad), dtype=torch.float32, device="cuda:0")
    with pytest.raises(chem.ChemError) as e:
        s.forward(X, out, path=2)
    assert e.value.code == -5
    s.forward(X, out, path=0)       # the library falls back to the GEMMs
    s.close()


def test_gradient_parity(torch, mechs):
    from chemgen.surrogate_data import split_params
    from oracle import surrogate as S
    from paper_2312_13513_amd import chem
    K, rows = 35, 640
    s, dims, flat = _surr(chem, mechs["M35"], K, seed=21)
    rng = np.random.default_rng(22)
    x = S.to_bf16(rng.normal(0, 1, (rows, K + 2)).astype(np.float32))
    Xb = np.zeros((rows, 64), dtype=np.uint16)
    Xb[:, :K + 2] = S.bf16_bits(x)
    tgt = rng.normal(0, 1, (rows, K)).astype(np.float32)
    X = torch.tensor(Xb.view(np.int16), device="cuda:0")
    loss = s.grad(X, _dev(torch, tgt, torch.float32))
    g = s.get_grads()
    params_bf = [(S.to_bf16(W.astype(np.float32)), b) for W, b in split_params(flat, dims)]
    out, cache = S.forward(params_bf, x)
    ref_loss = S.mse_loss(out, tgt.astype(np.float64))
    grads = S.backward(params_bf, cache, out, tgt.astype(np.float64))
    gg = split_params(g, dims)
    _say(f"[grad] loss gpu {loss:.6e} oracle {ref_loss:.6e}")
    assert abs(loss - ref_loss) <= 1e-2 * ref_loss
    for li, ((gW, gb), (rW, rb)) in enumerate(zip(gg, grads)):
        for name, a, r in (("W", gW, rW), ("b", gb, rb)):
            rel = np.linalg.norm(a - r) / np.linalg.norm(r)
            cos = float(np.sum(a * r) / (np.linalg.norm(a) * np.linalg.norm(r)))
            _say(f"    layer {li + 1} d{name}: rel-L2 {rel:.3e} cosine {cos:.6f}")
            assert rel <= 2e-2 and cos >= 0.999
    s.close()


def test_adam_parity(torch, mechs):
    from chemgen.surrogate_data import split_params
    from oracle import surrogate as S
    from paper_2312_13513_amd import chem
    K = 9
    s, dims, flat = _surr(chem, mechs["M9"], K, h=(64, 64, 64), seed=31)
    params = split_params(flat, dims)
    state = S.adam_state(params)
    rng = np.random.default_rng(32)
    for step in range(3):
        g = rng.normal(0, 1e-2, flat.size).astype(np.float32)
        g[rng.random(flat.size) < 0.05] = 0.0
        s.set_grads(g)
        s.adam(1e-3)
        S.adam_step(params, split_params(g, dims), state, 1e-3)
    got = split_params(s.get_params(), dims)
    worst = 0.0
    for (W, b), (rW, rb) in zip(got, params):
        for a, r in ((W, rW), (b, rb)):
            worst = max(worst, float(np.max(np.abs(a - r) / (np.abs(r) + 1e-3))))
    _say(f"[adam] worst |dp| / (|p| + lr) = {worst:.3e}")
    assert worst < 1e-5
    s.close()


def test_fit_norm_matches_numpy(torch, mechs, m35py):
    from chemgen.fields import zones128
    from oracle import surrogate as S
    from paper_2312_13513_amd import chem
    f = zones128(m35py, shape=(8, 8, 8))
    rng = np.random.default_rng(3)
    Yn = f.Y * np.exp(0.01 * rng.normal(size=f.Y.shape))
    s = chem.Surrogate(mechs["M35"], 64, 64, 64)
    s.fit_norm(_dev(torch, f.T), _dev(torch, f.p), _dev(torch, f.Y), _dev(torch, Yn), 1e-5)
    got = s.get_norm()
    ref = S.fit_norm(f.T, f.p, f.Y, Yn, 1e-5)
    assert np.all(np.abs(got - ref) <= 1e-12 * np.abs(ref) + 1e-300)
    s.close()


def _apply_case(m35py, rng, n=1536):
    from chemgen.fields import zones128
    f = zones128(m35py, shape=(16, 16, 8))
    idx = np.sort(rng.choice(f.n, size=n, replace=False))
    T, p, Y = f.T[idx], f.p[idx], np.ascontiguousarray(f.Y[:, idx])
    K = m35py.K
    W = m35py.molar_masses()
    # predictions: small random changes, element-conserving reaction moves,
    # zero changes and a few large ones, in z-score units of a synthetic norm
    mu_y = np.zeros(K)
    sig_y = np.full(K, 1e-4)
    yhat = rng.normal(0, 1, (n, K))
    for i in range(0, n, 3):
        r = m35py.reactions[int(rng.integers(len(m35py.reactions)))]
        nu = np.zeros(K)
        for k, c in r[0]:
            nu[k] -= c
        for k, c in r[1]:
            nu[k] += c
        yhat[i] = rng.normal(0, 1) * nu * W / np.max(np.abs(nu * W))
    yhat[1::7] = 0.0
    yhat[5::11] *= 300.0
    return T, p, Y, yhat.astype(np.float32), mu_y, sig_y


def test_apply_checks_parity(torch, mechs, m35py, om35):
    from oracle import surrogate as S
    from paper_2312_13513_amd import chem
    rng = np.random.default_rng(41)
    T, p, Y, yhat, mu_y, sig_y = _apply_case(m35py, rng)
    K, n = m35py.K, T.size
    s = chem.Surrogate(mechs["M35"], 64, 64, 64)
    norm = np.concatenate([np.zeros(K + 2), np.ones(K + 2), mu_y, sig_y, [1e-5]])
    s.set_norm(norm)
    out = np.zeros((n, s.nout_pad), dtype=np.float32)
    out[:, :K] = yhat
    Tg, Yg = _dev(torch, T), _dev(torch, Y)
    mask = torch.full((n,), -1, dtype=torch.int32, device="cuda:0")
    checks = chem.chem_surrogate_default_checks()
    s.apply(Tg, _dev(torch, p), Yg, _dev(torch, out, torch.float32), checks=checks, mask=mask)
    torch.cuda.synchronize()
    Tg, Yg, mk = Tg.cpu().numpy(), Yg.cpu().numpy(), mask.cpu().numpy()
    W = m35py.molar_masses()
    ok_ref = np.zeros(n, dtype=bool)
    Tr, Yr = T.copy(), Y.copy()
    for i in range(n):
        ok, Tn, Yn = S.apply_cell(om35, m35py.counts, W, T[i], Y[:, i], yhat[i].astype(np.float64),
                                  mu_y, sig_y)
        ok_ref[i] = ok
        Tr[i], Yr[:, i] = Tn, Yn
    _say(f"[apply] accepted gpu {np.sum(mk == 0)} oracle {ok_ref.sum()} of {n}")
    assert np.array_equal(mk == 0, ok_ref)
    assert 0 < ok_ref.sum() < n
    assert np.max(np.abs(Tg - Tr)) < 1e-8
    assert np.max(np.abs(Yg - Yr)) < 1e-14
    s.close()


def test_apply_unaligned_output_rows(torch, mechs, m35py):
    """A network output buffer that is not 16-byte aligned (a view one float
    into a larger allocation) takes the one-float-per-load decode; the result
    equals the vector-load decode of an aligned copy bit for bit."""
    from paper_2312_13513_amd import chem
    rng = np.random.default_rng(43)
    T, p, Y, yhat, mu_y, sig_y = _apply_case(m35py, rng)
    K, n = m35py.K, T.size
    s = chem.Surrogate(mechs["M35"], 64, 64, 64)
    s.set_norm(np.concatenate([np.zeros(K + 2), np.ones(K + 2), mu_y, sig_y, [1e-5]]))
    out = np.zeros((n, s.nout_pad), dtype=np.float32)
    out[:, :K] = yhat
    aligned = _dev(torch, out, torch.float32)
    big = torch.zeros(n * s.nout_pad + 1, dtype=torch.float32, device="cuda:0")
    shifted = big[1:].view(n, s.nout_pad)
    shifted.copy_(aligned)
    assert aligned.data_ptr() % 16 == 0 and shifted.data_ptr() % 16 == 4
    res = []
    for o in (aligned, shifted):
        Tg, Yg = _dev(torch, T), _dev(torch, Y)
        mask = torch.full((n,), -1, dtype=torch.int32, device="cuda:0")
        s.apply(Tg, _dev(torch, p), Yg, o, checks=chem.chem_surrogate_default_checks(), mask=mask)
        torch.cuda.synchronize()
        res.append((Tg.cpu().numpy(), Yg.cpu().numpy(), mask.cpu().numpy()))
    _say(f"[apply unaligned] accepted {np.sum(res[0][2] == 0)} of {n}")
    for a, b in zip(*res):
        assert np.array_equal(a, b)
    assert 0 < np.sum(res[0][2] == 0) < n
    s.close()


def _train_set(torch, chem, mech, mpy, n_flame, n_traj, traj_steps, dt, seed):
    """Training states and their successors over dt, labelled by the GPU
    integrator (trajectory states are recorded step by step)."""
    from chemgen.surrogate_data import flame_like_states, trajectory_starts
    T1, p1, Y1 = flame_like_states(mpy, n_flame, seed)
    T2, p2, Y2 = trajectory_starts(mpy, n_traj, seed + 1)
    Ts, ps, Ys = [T1], [p1], [Y1]
    Tt, pt, Yt = _dev(torch, T2), _dev(torch, p2), _dev(torch, Y2)
    for _ in range(traj_steps - 1):
        mech.integrate(Tt, pt, Yt, dt)
        Ts.append(Tt.cpu().numpy().copy())
        ps.append(p2)
        Ys.append(Yt.cpu().numpy().copy())
    T = np.concatenate(Ts)
    p = np.concatenate(ps)
    Y = np.ascontiguousarray(np.concatenate(Ys, axis=1))
    Td, pd, Yd = _dev(torch, T), _dev(torch, p), _dev(torch, Y)
    Yn = Yd.clone()
    Tn = Td.clone()
    mech.integrate(Tn, pd, Yn, dt)
    return Td, pd, Yd, Yn


def test_training_gain_over_untrained(torch, mechs, mech_dir, tmp_path):
    """Train on integrator-labelled states of the 9-species mechanism, then
    serve a held-out flame field: the trained network keeps most cells within
    the checks and every cell within 5 K of the FP64 oracle, with several
    times less error than the untrained network (same normalisation, initial
    weights, same checks and fallback).  The trained weights survive a
    save/load round trip."""
    from chemgen.fields import flame_field
    from chemgen.mechanism import read_mechanism
    from chemgen.surrogate_data import epoch_orders, init_params, network_dims
    import oracle
    from paper_2312_13513_amd import chem
    mpy = read_mechanism(str(mech_dir / "M9.mech"))
    mech = mechs["M9"]
    dt, K = 1e-6, mpy.K
    h = (128, 128, 64)
    Td, pd, Yd, Yn = _train_set(torch, chem, mech, mpy, 24576, 256, 32, dt, seed=71)
    n = Td.shape[0]
    s = chem.Surrogate(mech, *h)
    init = init_params(network_dims(K, *h), 72)
    s.set_params(init)
    s.fit_norm(Td, pd, Yd, Yn, dt)
    epochs = 12
    order = _dev(torch, epoch_orders(n, epochs, 73), torch.int32)
    losses = s.train(Td, pd, Yd, Yn, epochs=epochs, batch=1024, lr0=1e-3, lr1=1e-5, order=order)
    _say(f"[train] n={n} loss per epoch {np.array2string(losses, precision=4)}")
    assert np.all(np.isfinite(losses)) and losses[-1] < 0.5 * losses[0]
    # held-out field with the same mixture
    f = flame_field(mpy, (24, 24, 24), seed=74, dt=dt, name="heldout", mech_name="M9", mix_seed=7)
    om = oracle.OracleMech(str(mech_dir / "M9.mech"))
    To, Yo, _, _, _ = om.integrate(f.T, f.p, f.Y, dt)

    def serve(surr):
        T, Y = _dev(torch, f.T), _dev(torch, f.Y)
        mask = torch.zeros(f.n, dtype=torch.int32, device="cuda:0")
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda:0")
        surr.infer(T, _dev(torch, f.p), Y, dt, mask=mask, fallback_count=cnt)
        torch.cuda.synchronize()
        return T.cpu().numpy(), Y.cpu().numpy(), mask.cpu().numpy(), int(cnt.item())

    Tt, Yt, mt, ct = serve(s)
    path = str(tmp_path / "m9.surr")
    s.save(path)
    s2 = chem.Surrogate.load(mech, path)
    assert np.array_equal(s2.get_params(), s.get_params())
    assert np.array_equal(s2.get_norm(), s.get_norm())
    Tl, Yl, ml, cl = serve(s2)
    assert np.array_equal(Tl, Tt) and np.array_equal(Yl, Yt) and np.array_equal(ml, mt)
    s2.close()
    u = chem.Surrogate(mech, *h)
    u.set_params(init)
    u.set_norm(s.get_norm())
    Tu, Yu, mu, cu = serve(u)
    dT_t = np.abs(Tt - To)
    dT_u = np.abs(Tu - To)
    _say(f"[serve] trained: fallback {ct}/{f.n}, max|dT| {dT_t.max():.3f} K; "
         f"untrained: fallback {cu}/{f.n}, max|dT| {dT_u.max():.3f} K")
    _say(f"[serve] mean|dT| trained {dT_t.mean():.4f} K untrained {dT_u.mean():.4f} K")
    assert ct == int(mt.sum()) and cu == int(mu.sum())
    assert ct <= cu and ct <= 0.5 * f.n
    assert dT_t.max() <= 5.0
    # what training buys at the same checks: a several times smaller error
    assert 3.0 * dT_t.max() <= dT_u.max() and 3.0 * dT_t.mean() <= dT_u.mean()
    s.close()
    u.close()


def test_all_fallback_is_bitwise_plain(torch, mechs, m35py):
    """With checks no cell can pass, the surrogate path is the integrator:
    results are bitwise those of chem_integrate on the same cells."""
    from chemgen.fields import zones128
    from paper_2312_13513_amd import chem
    f = zones128(m35py, shape=(8, 8, 8))
    K = m35py.K
    rng = np.random.default_rng(81)
    s, dims, flat = _surr(chem, mechs["M35"], K, h=(64, 64, 64), seed=82)
    s.set_norm(_synthetic_norm(f.T, f.p, f.Y, K, rng))
    checks = chem.chem_surrogate_default_checks()
    checks.T_in_max = 0.0
    T1, Y1 = _dev(torch, f.T), _dev(torch, f.Y)
    pt = _dev(torch, f.p)
    mask = torch.zeros(f.n, dtype=torch.int32, device="cuda:0")
    st = torch.full((f.n,), -1, dtype=torch.int32, device="cuda:0")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    s.infer(T1, pt, Y1, f.dt, checks=checks, mask=mask, status=st, fallback_count=cnt)
    T2, Y2 = _dev(torch, f.T), _dev(torch, f.Y)
    st2 = torch.full((f.n,), -1, dtype=torch.int32, device="cuda:0")
    mechs["M35"].integrate(T2, pt, Y2, f.dt, status=st2)
    torch.cuda.synchronize()
    assert int(cnt.item()) == f.n and bool(torch.all(mask == 1))
    assert torch.equal(T1, T2) and torch.equal(Y1, Y2) and torch.equal(st, st2)
    s.close()


def test_infer_rejects_other_dt_and_bad_args(torch, mechs, m35py):
    from paper_2312_13513_amd import chem
    s = chem.Surrogate(mechs["M35"], 64, 64, 64)
    T = torch.full((4,), 1000.0, dtype=torch.float64, device="cuda:0")
    Y = torch.full((35, 4), 1 / 35, dtype=torch.float64, device="cuda:0")
    with pytest.raises(chem.ChemError):
        s.infer(T, T, Y, 1e-5)                      # no normalisation yet
    norm = np.concatenate([np.zeros(37), np.ones(37), np.zeros(35), np.ones(35) * 1e-4, [1e-5]])
    s.set_norm(norm)
    with pytest.raises(chem.ChemError):
        s.infer(T, T, Y, 2e-5)                      # other flow step
    with pytest.raises(chem.ChemError):
        s.set_params(np.zeros(3, dtype=np.float32))  # wrong length
    with pytest.raises(chem.ChemError):
        chem.Surrogate(mechs["M35"], 100, 64, 64)   # width not a multiple of 64
    s.infer(T[:0], T[:0], Y[:, :0], 1e-5)           # zero cells: no-op
    s.close()
