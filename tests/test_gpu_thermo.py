"""GPU parity of the field property kernels (Section 3.1, the Thermo class;
the mixture-averaged transport of Section 2) through the C ABI, against the
oracle on the same seeded inputs.

Bars (u = 2^-53):
* mixture h and cp: each is a sum of K products of a polynomial value and a
  mass fraction, rounded differently on the two sides (FMA chains on the
  GPU): within 1e-13 of the sum of the magnitudes of the terms.
* T from h: both sides stop once a Newton step is below 1e-10 K, after
  which the iterate is within far less than that of the root of their own
  h(T); the two roots differ by the rounding of h, about 1e-16 of the
  gross enthalpy over cp, below 1e-10 K.  Bar |dT| <= 1e-9 K, cp within
  1e-11 relative, the step counts within one (a last step that lands near
  1e-10 K may fall on either side).  Non-convergence is NaN on both sides.
* viscosity and conductivity: sums of K positive terms each a few roundings
  apart (K <= 64): within 1e-12 relative.
* diffusion: the same, plus the cancellation in 1 - y_k, whose operands
  carry a few u: within 1e-12 + 1e-15 / (1 - y_k) relative."""
import numpy as np
import pytest

from test_gpu_integrate import _say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


def _mech(name):
    from chemgen.mechanism import make_mechanism, standard_mechanism
    if name == "K64":
        return make_mechanism(seed=78, K=64, R=150, E=4)
    if name.startswith("K") and name[1:].isdigit():
        k = int(name[1:])
        return make_mechanism(seed=70 + k, K=k, R=max(12, 2 * k), E=3 if k < 30 else 4)
    return standard_mechanism(name)


def _open(tmp_path, name):
    from paper_2312_13513_amd import chem
    mech = _mech(name)
    path = str(tmp_path / f"{name}.mech")
    mech.write(path)
    return mech, chem.Mechanism(path), path


def _state(K, n, seed):
    """T over 300-3000 K (both NASA ranges), p 0.5-4 atm, Dirichlet mass
    fractions with exact zeros, tiny negatives, unnormalised cells and
    pure-species cells."""
    rng = np.random.default_rng(seed)
    T = rng.uniform(300.0, 3000.0, n)
    p = rng.uniform(0.5, 4.0, n) * 101325.0
    Y = rng.dirichlet(np.full(K, 0.6), n).T.copy()
    Y[rng.integers(0, K, n // 5), rng.integers(0, n, n // 5)] = 0.0
    neg = rng.integers(0, n, n // 10)
    Y[rng.integers(0, K, neg.size), neg] = -1e-12
    Y[:, : n // 20] *= 1.0 + 1e-6
    for i in range(min(K, n // 50)):
        Y[:, n - 1 - i] = 0.0
        Y[i, n - 1 - i] = 1.0
    return T, p, Y


def _dev(torch, a, ld=None, dtype=None):
    """Device copy; a 2-D array gets leading dimension ld >= its columns."""
    dt = dtype or torch.float64
    if a.ndim == 1 or ld is None:
        return torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda:0")
    out = torch.full((a.shape[0], ld), float("nan"), dtype=dt, device="cuda:0")
    out[:, : a.shape[1]] = torch.tensor(a, dtype=dt, device="cuda:0")
    return out


def _transport_check(tag, mech, fits, T, p, Y, mu, lam, D):
    from oracle import transport as TR
    W = mech.molar_masses()
    mu_o, lam_o, D_o = TR.transport(*fits, W, T, p, Y)
    y, _ = TR.composition(W, Y)
    e_mu = np.abs(mu / mu_o - 1).max()
    e_lam = np.abs(lam / lam_o - 1).max()
    with np.errstate(divide="ignore"):
        bar = 1e-12 + 1e-15 / np.maximum(1.0 - y, 1e-300)
    e_D = (np.abs(D - D_o) / (np.abs(D_o) * bar)).max()
    _say(f"{tag}: mu {e_mu:.2e}  lam {e_lam:.2e}  D {e_D:.3f} of bar")
    assert e_mu <= 1e-12 and e_lam <= 1e-12 and e_D <= 1.0
    assert np.all(np.isfinite(mu)) and np.all(np.isfinite(D))


@pytest.mark.parametrize("name", ["K6", "M9", "H2R", "K11", "K12", "K14", "K16", "K18", "CH4R", "M35", "K64"])
def test_transport_parity(torch, tmp_path, name):
    """Wilke viscosity, Mathur conductivity and mixture-averaged diffusion
    over 3,001 cells (several blocks and a ragged tail) with padded leading
    dimensions, for K = 6 .. 64: every kernel bound from 9 to 64, the
    unrolled bounds (9, 12, 16, 20) both with K equal to the bound and with
    padding."""
    from chemgen.transport import transport_fits
    mech, m, _ = _open(tmp_path, name)
    fits = transport_fits(mech, 21)
    m.set_transport(*fits)
    n = 3001
    T, p, Y = _state(mech.K, n, 31)
    Td, pd, Yd = _dev(torch, T), _dev(torch, p), _dev(torch, Y, n + 7)
    mu = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda:0")
    lam = torch.full_like(mu, float("nan"))
    D = torch.full((mech.K, n + 3), float("nan"), dtype=torch.float64, device="cuda:0")
    m.transport(Td, pd, Yd, mu, lam, D)
    torch.cuda.synchronize()
    Dh = D.cpu().numpy()
    assert np.all(np.isnan(Dh[:, n:])), "D written beyond ncells"
    _transport_check(f"transport {name}", mech, fits, T, p, Y, mu.cpu().numpy(), lam.cpu().numpy(), Dh[:, :n])
    # the split calls (viscosity and conductivity only; diffusion only) give the same bits
    mu2, lam2, D2 = torch.zeros_like(mu), torch.zeros_like(lam), torch.zeros_like(D)
    m.transport(Td, pd, Yd, mu2, lam2, None)
    m.transport(Td, pd, Yd, None, None, D2)
    torch.cuda.synchronize()
    assert torch.equal(mu2, mu) and torch.equal(lam2, lam) and torch.equal(D2[:, :n], D[:, :n])
    m.close()


@pytest.mark.parametrize("name", ["K6", "M9", "H2R", "K14", "K18", "CH4R", "M35", "K64"])
def test_h_cp_and_T_from_h_parity(torch, tmp_path, name, oracle_lib):
    """Mixture h and cp at T, then T back from h by Newton from guesses
    150 K away (across the NASA range boundary for some cells), with cp and
    the step counts; cells with an unreachable enthalpy end in NaN with
    max_iter + 1 steps on both sides."""
    from oracle import transport as TR
    mech, m, path = _open(tmp_path, name)
    om = oracle_lib.OracleMech(path)
    n = 1501
    T, _, Y = _state(mech.K, n, 41)
    Y = np.abs(Y)
    Td, Yd = _dev(torch, T), _dev(torch, Y, n + 5)
    h = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda:0")
    cp = torch.full_like(h, float("nan"))
    m.mixture_h_cp(Td, Yd, h, cp)
    torch.cuda.synchronize()
    h_g, cp_g = h.cpu().numpy(), cp.cpu().numpy()
    R_U = 8.31446261815324
    W = mech.molar_masses()
    gross_h = np.zeros(n)
    gross_cp = np.zeros(n)
    h_o = np.zeros(n)
    cp_o = np.zeros(n)
    for i in range(n):
        cpR, hRT, _ = om.thermo(T[i])
        gross_h[i] = np.sum(np.abs(Y[:, i] * R_U * T[i] * hRT / W))
        gross_cp[i] = np.sum(np.abs(Y[:, i] * R_U * cpR / W))
        h_o[i] = om.enthalpy(T[i], Y[:, i])
        cp_o[i] = np.sum(Y[:, i] * cpR * R_U / W)
    e_h = (np.abs(h_g - h_o) / gross_h).max()
    e_cp = (np.abs(cp_g - cp_o) / gross_cp).max()
    _say(f"h/cp {name}: h {e_h:.2e}  cp {e_cp:.2e} of the gross sums")
    assert e_h <= 1e-13 and e_cp <= 1e-13
    # T from the oracle's enthalpy (no input from the GPU side)
    guess = np.where(T < 1650.0, T + 150.0, T - 150.0)
    hb = h_o.copy()
    bad = np.arange(0, n, 97)
    hb[bad] += 1e9            # beyond h(3500 K): no root in the clamp range
    Tg = _dev(torch, guess)
    cp2 = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda:0")
    its = torch.full((n,), -1, dtype=torch.int32, device="cuda:0")
    m.T_from_h(_dev(torch, hb), Yd, Tg, cp2, its, max_iter=20, tol=1e-10)
    torch.cuda.synchronize()
    T_o, cp_oo, it_o = TR.thermo_field(om, hb, Y, guess)
    T_g, cp_gg, it_g = Tg.cpu().numpy(), cp2.cpu().numpy(), its.cpu().numpy()
    ok = np.isfinite(T_o)
    assert np.array_equal(ok, np.isfinite(T_g)) and not ok[bad].any()
    assert np.all(it_g[~ok] == 21) and np.all(np.isnan(cp_gg[~ok]))
    dT = np.abs(T_g[ok] - T_o[ok]).max()
    e_c = np.abs(cp_gg[ok] / cp_oo[ok] - 1).max()
    d_it = np.abs(it_g[ok] - it_o[ok]).max()
    _say(f"T_from_h {name}: |dT| {dT:.2e} K  cp {e_c:.2e}  steps within {d_it}  "
         f"(mean steps {it_g[ok].mean():.2f})")
    assert dT <= 1e-9 and e_c <= 1e-11 and d_it <= 1
    assert np.abs(T_g[ok] - T[ok]).max() <= 1e-8
    m.close()


def test_property_edge_cases(torch, tmp_path):
    """No-op on zero cells; argument errors; a mechanism beyond 64 species
    is refused by the property kernels."""
    from chemgen.mechanism import make_mechanism
    from chemgen.transport import transport_fits
    from paper_2312_13513_amd import chem
    mech, m, _ = _open(tmp_path, "M9")
    T, p, Y = _state(mech.K, 300, 5)
    Td, pd, Yd = _dev(torch, T), _dev(torch, p), _dev(torch, Y)
    mu, lam = torch.zeros(300, dtype=torch.float64, device="cuda:0"), torch.zeros(300, dtype=torch.float64,
                                                                                   device="cuda:0")
    D = torch.zeros((mech.K, 300), dtype=torch.float64, device="cuda:0")
    with pytest.raises(chem.ChemError, match="chem_set_transport"):
        m.transport(Td, pd, Yd, mu, lam, D)
    fits = transport_fits(mech, 3)
    bad = fits[2].copy()
    bad[0, 1, 2] += 1e-9
    with pytest.raises(chem.ChemError, match="symmetric"):
        m.set_transport(fits[0], fits[1], bad)
    m.set_transport(*fits)
    m.transport(Td, pd, Yd, mu, lam, D, ncells=0)
    with pytest.raises(chem.ChemError, match="together"):
        m.transport(Td, pd, Yd, mu, None, D)
    with pytest.raises(chem.ChemError, match="max_iter"):
        m.T_from_h(Td, Yd, Td.clone(), max_iter=0)
    with pytest.raises(chem.ChemError, match="tol"):
        m.T_from_h(Td, Yd, Td.clone(), tol=0.0)
    m.T_from_h(Td, Yd, Td.clone(), ncells=0)
    m.mixture_h_cp(Td, Yd, None, None, ncells=0)
    m.close()
    big = make_mechanism(seed=79, K=65, R=150, E=4)
    path = str(tmp_path / "K65.mech")
    big.write(path)
    m65 = chem.Mechanism(path)
    Y65 = torch.full((65, 10), 1.0 / 65, dtype=torch.float64, device="cuda:0")
    T65 = torch.full((10,), 1000.0, dtype=torch.float64, device="cuda:0")
    with pytest.raises(chem.ChemError, match="64 species"):
        m65.mixture_h_cp(T65, Y65, T65.clone(), None)
    m65.close()


def test_tgv_share_full_size_sampled(torch, tmp_path, oracle_lib):
    """The benchmark's workload at full size (4,194,304 cells of the
    9-species mechanism, one GPU's share of the 256^3 TGV mesh), in the
    benchmark's calls: h from T on the GPU, T back from h from the previous
    step's guess, then transport; checked on 2,000 seeded cells against the
    oracle (whose T from h starts at the same guess from the oracle's own h)."""
    from chemgen.fields import newton_guess, seeded_sample, tgv_share
    from chemgen.transport import transport_fits
    from oracle import transport as TR
    mech, m, path = _open(tmp_path, "M9")
    om = oracle_lib.OracleMech(path)
    f = tgv_share(mech)
    n = f.n
    fits = transport_fits(mech, 9)
    m.set_transport(*fits)
    guess = newton_guess(f.T, 12)
    Td, pd, Yd = _dev(torch, f.T), _dev(torch, f.p), _dev(torch, f.Y)
    h = torch.empty(n, dtype=torch.float64, device="cuda:0")
    m.mixture_h_cp(Td, Yd, h, None)
    Tn = _dev(torch, guess)
    cp = torch.empty_like(h)
    its = torch.empty(n, dtype=torch.int32, device="cuda:0")
    m.T_from_h(h, Yd, Tn, cp, its)
    mu, lam = torch.empty_like(h), torch.empty_like(h)
    D = torch.empty((mech.K, n), dtype=torch.float64, device="cuda:0")
    m.transport(Tn, pd, Yd, mu, lam, D)
    torch.cuda.synchronize()
    idx = seeded_sample(n, 2000, 13)
    Ts, Ys, ps = f.T[idx], f.Y[:, idx], f.p[idx]
    h_o = np.array([om.enthalpy(Ts[j], Ys[:, j]) for j in range(idx.size)])
    T_o, cp_o, it_o = TR.thermo_field(om, h_o, Ys, guess[idx])
    Tg = Tn.cpu().numpy()[idx]
    assert np.abs(Tg - T_o).max() <= 1e-9
    assert np.abs(cp.cpu().numpy()[idx] / cp_o - 1).max() <= 1e-11
    assert np.abs(its.cpu().numpy()[idx] - it_o).max() <= 1
    _say(f"tgv_share: mean Newton steps {its.float().mean().item():.2f}, max {its.max().item()}")
    _transport_check("tgv_share transport", mech, fits, Tg, ps, Ys, mu.cpu().numpy()[idx], lam.cpu().numpy()[idx],
                     D.cpu().numpy()[:, idx])
    m.close()
