"""GPU parity of the paper's per-species network variant (Section 2: one
network per species, GELU, Adam) run as grouped BF16 MFMA products, through
the C ABI, against the FP64 oracle's forward_species / backward_species.

Bars as for the single network (tests/test_gpu_surrogate.py): every hidden
activation equals the oracle's BF16 rounding of GELU(u) from the GPU's own
BF16 inputs, except within the FP32 accumulation error of a rounding
boundary; each output within its accumulation error; gradients by norms
(rel-L2 <= 2e-2, cosine >= 0.999 per layer and network)."""
import numpy as np
import pytest

from test_gpu_integrate import _say
from test_gpu_surrogate import GELU_LIP, _bf16_vals, _dev, _train_set, mechs, torch  # noqa: F401

pytestmark = pytest.mark.gpu

GELU_REL = 2.5e-5


def _species_surr(chem, mech, K, h, seed):
    from chemgen.surrogate_data import init_species_params, species_network_dims
    s = chem.Surrogate(mech, *h, per_species=True)
    flat = init_species_params(K, h, seed)
    # non-zero biases exercise the bias epilogues
    rng = np.random.default_rng(seed + 100)
    per = sum(a * b + b for a, b in species_network_dims(K, *h))
    o = 0
    for g in range(K):
        for fi, fo in species_network_dims(K, *h):
            o += fi * fo
            flat[o:o + fo] = rng.normal(0, 0.05, fo).astype(np.float32)
            o += fo
    assert o == K * per == flat.size, (o, K * per, flat.size)
    assert s.nparams == flat.size and s.groups == K, (s.nparams, flat.size, s.groups)
    s.set_params(flat)
    return s, flat


@pytest.mark.parametrize("rows,h", [(1, (128, 64, 64)), (63, (128, 64, 64)), (2050, (128, 64, 64)),
                                    (257, (100, 72, 40))])
def test_species_forward_parity(torch, mechs, rows, h):
    """K = 9 networks: the per-layer BF16 activations of every species' block
    against the oracle, and each species' output; widths that are not
    multiples of 64 are padded with units that stay exactly zero."""
    from chemgen.surrogate_data import split_species_params
    from oracle import surrogate as S
    from paper_2312_13513_amd import chem
    K = 9
    hp = [(w + 63) // 64 * 64 for w in h]
    s, flat = _species_surr(chem, mechs["M9"], K, h, 41)
    rng = np.random.default_rng(rows + 5)
    x = S.to_bf16(rng.normal(0, 1, (rows, K + 2)).astype(np.float32))
    Xb = np.zeros((rows, 64), dtype=np.uint16)
    Xb[:, :K + 2] = S.bf16_bits(x)
    X = torch.tensor(Xb.view(np.int16), device="cuda:0")
    out = torch.zeros((rows, s.nout_pad), dtype=torch.float32, device="cuda:0")
    s.forward(X, out, path=0)
    H = [torch.zeros((rows, w), dtype=torch.int16, device="cuda:0") for w in (s.h1, s.h2, s.h3)]
    out_t = torch.full((rows, s.nout_pad), -9.0, dtype=torch.float32, device="cuda:0")
    s.forward_trace(X, *H, out_t)
    torch.cuda.synchronize()
    assert torch.equal(out, out_t)
    Hh = [_bf16_vals(t) for t in H]
    got_out = out.cpu().numpy()
    nets = split_species_params(flat, K, h)
    n_act = n_flip = 0
    worst = 0.0
    for g in range(K):
        params_bf = [(S.to_bf16(W.astype(np.float32)), b) for W, b in nets[g]]
        hin = x
        for li in range(3):
            W, b = params_bf[li]
            u = hin @ W.T + b
            tol_u = (W.shape[1] + 1) * 2.0 ** -24 * (np.abs(hin) @ np.abs(W).T + np.abs(b))
            gl = S.gelu(u)
            tol = 2.0 * (GELU_LIP * tol_u + GELU_REL * np.abs(gl)) + 1e-37
            got = Hh[li][:, g * hp[li]:g * hp[li] + h[li]]
            assert np.all(Hh[li][:, g * hp[li] + h[li]:(g + 1) * hp[li]] == 0.0)
            exact = S.to_bf16(gl)
            lo, hi = S.to_bf16(gl - tol), S.to_bf16(gl + tol)
            flip = got != exact
            n_act += got.size
            n_flip += int(flip.sum())
            assert np.all(~flip | ((got >= lo) & (got <= hi) & (lo != hi))), (g, li)
            hin = got
        W, b = params_bf[3]
        ref = (hin @ W.T + b)[:, 0]
        tol = 2.0 * (W.shape[1] + 1) * 2.0 ** -24 * ((np.abs(hin) @ np.abs(W).T)[:, 0] + np.abs(b[0])) + 1e-30
        err = np.abs(got_out[:, g] - ref)
        worst = max(worst, float((err / tol).max()))
        assert np.all(err <= tol), g
    _say(f"[species forward rows={rows}] {n_act} activations, {n_flip} rounding flips; "
         f"output max err/tol {worst:.3f}")
    assert n_flip <= max(2, 0.02 * n_act)
    assert np.all(got_out[:, K:] == 0.0)
    s.close()


@pytest.mark.parametrize("h,rows", [((128, 64, 64), 640), ((512, 72, 64), 256)])
def test_species_gradient_parity(torch, mechs, h, rows):
    """Gradients of all K networks by norms; the second case has a first
    layer of 9 x 512 = 4,608 units in all, wider than any single network,
    whose partial bias gradients the training buffers must hold."""
    from chemgen.surrogate_data import split_species_params
    from oracle import surrogate as S
    from paper_2312_13513_amd import chem
    K = 9
    s, flat = _species_surr(chem, mechs["M9"], K, h, 51)
    rng = np.random.default_rng(52)
    x = S.to_bf16(rng.normal(0, 1, (rows, K + 2)).astype(np.float32))
    Xb = np.zeros((rows, 64), dtype=np.uint16)
    Xb[:, :K + 2] = S.bf16_bits(x)
    tgt = rng.normal(0, 1, (rows, K)).astype(np.float32)
    X = torch.tensor(Xb.view(np.int16), device="cuda:0")
    loss = s.grad(X, _dev(torch, tgt, torch.float32))
    gg = split_species_params(s.get_grads(), K, h)
    nets = [[(S.to_bf16(W.astype(np.float32)), b) for W, b in net] for net in split_species_params(flat, K, h)]
    out, caches = S.forward_species(nets, x)
    ref_loss = S.mse_loss(out, tgt.astype(np.float64))
    ref = S.backward_species(nets, caches, out, tgt.astype(np.float64))
    _say(f"[species grad] loss gpu {loss:.6e} oracle {ref_loss:.6e}")
    assert abs(loss - ref_loss) <= 1e-2 * ref_loss
    worst_rel, worst_cos = 0.0, 1.0
    for g in range(K):
        for li in range(4):
            for a, r in ((gg[g][li][0], ref[g][li][0]), (gg[g][li][1], ref[g][li][1])):
                rel = np.linalg.norm(a - r) / np.linalg.norm(r)
                cos = float(np.sum(a * r) / (np.linalg.norm(a) * np.linalg.norm(r)))
                worst_rel, worst_cos = max(worst_rel, rel), min(worst_cos, cos)
    _say(f"    worst rel-L2 {worst_rel:.3e}, worst cosine {worst_cos:.6f} over {K} networks x 4 layers")
    assert worst_rel <= 2e-2 and worst_cos >= 0.999
    s.close()


def test_species_training_and_serving(torch, mechs, mech_dir, tmp_path):
    """Per-species networks train (loss falls by half in 8 epochs), serve a
    held-out field through the same checks and fallback within 5 K of the
    FP64 oracle, and are refused by the one-network weights file and the
    fused kernel."""
    from chemgen.fields import flame_field
    from chemgen.mechanism import read_mechanism
    from chemgen.surrogate_data import epoch_orders, init_species_params
    import oracle
    from paper_2312_13513_amd import chem
    mpy = read_mechanism(str(mech_dir / "M9.mech"))
    mech = mechs["M9"]
    dt, K, h = 1e-6, mpy.K, (128, 64, 64)
    Td, pd, Yd, Yn = _train_set(torch, chem, mech, mpy, 16384, 256, 32, dt, seed=81)
    n = Td.shape[0]
    s = chem.Surrogate(mech, *h, per_species=True)
    s.set_params(init_species_params(K, h, 82))
    s.fit_norm(Td, pd, Yd, Yn, dt)
    epochs = 8
    order = _dev(torch, epoch_orders(n, epochs, 83), torch.int32)
    losses = s.train(Td, pd, Yd, Yn, epochs=epochs, batch=1024, lr0=1e-3, lr1=1e-5, order=order)
    _say(f"[species train] n={n} loss per epoch {np.array2string(losses, precision=4)}")
    assert np.all(np.isfinite(losses)) and losses[-1] < 0.5 * losses[0]
    f = flame_field(mpy, (20, 20, 20), seed=84, dt=dt, name="heldout", mech_name="M9", mix_seed=7)
    om = oracle.OracleMech(str(mech_dir / "M9.mech"))
    To, _, _, _, _ = om.integrate(f.T, f.p, f.Y, dt)
    T, Y = _dev(torch, f.T), _dev(torch, f.Y)
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    s.infer(T, _dev(torch, f.p), Y, dt, fallback_count=cnt)
    torch.cuda.synchronize()
    dT = np.abs(T.cpu().numpy() - To)
    _say(f"[species serve] fallback {int(cnt.item())}/{f.n}, max|dT| {dT.max():.3f} K, mean {dT.mean():.4f} K")
    assert dT.max() <= 5.0
    with pytest.raises(chem.ChemError, match="per-species"):
        s.save(str(tmp_path / "x.surr"))
    X = torch.zeros((4, 64), dtype=torch.int16, device="cuda:0")
    out = torch.zeros((4, s.nout_pad), dtype=torch.float32, device="cuda:0")
    with pytest.raises(chem.ChemError, match="one network"):
        s.forward(X, out, path=2)
    s.close()


def test_species_full_size_sampled(torch, mechs):
    """The benchmark's configuration: 9 networks of 1600 / 800 / 400 units
    (padded to 1600 / 832 / 448) on 262,144 rows (the flame64 field's size,
    128 x 128 tiles).  Rows are independent and every output element sees the
    same MFMA sequence whatever the tile, so 96 seeded rows of the full-size
    output must equal, bit for bit, a 96-row forward of those rows (64 x 64
    tiles); that small forward is checked layer by layer against the
    oracle as in test_species_forward_parity."""
    from chemgen.fields import seeded_sample
    from chemgen.surrogate_data import split_species_params
    from oracle import surrogate as S
    from paper_2312_13513_amd import chem
    K, h, rows = 9, (1600, 800, 400), 262144
    hp = [(w + 63) // 64 * 64 for w in h]
    s, flat = _species_surr(chem, mechs["M9"], K, h, 61)
    rng = np.random.default_rng(62)
    x = S.to_bf16(rng.normal(0, 1, (rows, K + 2)).astype(np.float32))
    Xb = np.zeros((rows, 64), dtype=np.uint16)
    Xb[:, :K + 2] = S.bf16_bits(x)
    X = torch.tensor(Xb.view(np.int16), device="cuda:0")
    out = torch.zeros((rows, s.nout_pad), dtype=torch.float32, device="cuda:0")
    s.forward(X, out)
    idx = seeded_sample(rows, 96, 63)
    Xs = X[torch.tensor(idx, device="cuda:0")].contiguous()
    H = [torch.zeros((idx.size, K * w), dtype=torch.int16, device="cuda:0") for w in hp]
    out_s = torch.zeros((idx.size, s.nout_pad), dtype=torch.float32, device="cuda:0")
    s.forward_trace(Xs, *H, out_s)
    torch.cuda.synchronize()
    full = out.cpu().numpy()[idx]
    small = out_s.cpu().numpy()
    assert np.array_equal(full, small), "full-size rows differ from the same rows run alone"
    Hh = [_bf16_vals(t) for t in H]
    nets = split_species_params(flat, K, h)
    xs = x[idx]
    n_act = n_flip = 0
    for g in range(K):
        params_bf = [(S.to_bf16(W.astype(np.float32)), b) for W, b in nets[g]]
        hin = xs
        for li in range(3):
            W, b = params_bf[li]
            u = hin @ W.T + b
            tol_u = (W.shape[1] + 1) * 2.0 ** -24 * (np.abs(hin) @ np.abs(W).T + np.abs(b))
            gl = S.gelu(u)
            tol = 2.0 * (GELU_LIP * tol_u + GELU_REL * np.abs(gl)) + 1e-37
            got = Hh[li][:, g * hp[li]:g * hp[li] + h[li]]
            exact = S.to_bf16(gl)
            lo, hi = S.to_bf16(gl - tol), S.to_bf16(gl + tol)
            flip = got != exact
            n_act += got.size
            n_flip += int(flip.sum())
            assert np.all(~flip | ((got >= lo) & (got <= hi) & (lo != hi))), (g, li)
            hin = got
        W, b = params_bf[3]
        ref = (hin @ W.T + b)[:, 0]
        tol = 2.0 * (W.shape[1] + 1) * 2.0 ** -24 * ((np.abs(hin) @ np.abs(W).T)[:, 0] + np.abs(b[0])) + 1e-30
        assert np.all(np.abs(small[:, g] - ref) <= tol), g
    _say(f"[species full size] {rows} rows, {idx.size} sampled: {n_act} activations, {n_flip} rounding flips")
    assert n_flip <= max(2, 0.02 * n_act)
    s.close()
