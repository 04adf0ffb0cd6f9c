"""Pins of the thermo/transport field oracle (paper Section 3.1, the Thermo
class; the mixture-averaged transport model named in Section 2) against
facts other than its own formulas: the symmetry identity of Wilke's factor,
single-species and identical-species limits, hand-derived binary closed
forms, invariance under species reordering and pressure scaling, the
kinetic-theory values the seeded fits approximate, and the enthalpy round
trip with cp as the derivative of h."""
import numpy as np
import pytest

from chemgen.mechanism import standard_mechanism
from chemgen.transport import T_FIT, transport_fits
from oracle import transport as TR


def _state(K, n, seed, tlo=400.0, thi=2800.0):
    rng = np.random.default_rng(seed)
    T = rng.uniform(tlo, thi, n)
    p = rng.uniform(0.5e5, 4e5, n)
    Y = rng.dirichlet(np.full(K, 0.7), n).T.copy()
    return T, p, Y


@pytest.fixture(scope="module")
def m9fits():
    m = standard_mechanism("M9")
    return m, transport_fits(m, 11)


def test_wilke_factor_identity():
    """Phi_jk = (mu_j / mu_k) (W_k / W_j) Phi_kj for any pair (Bird, Stewart
    and Lightfoot's identity, exact for Wilke's form), and Phi_kk = 1.  A
    swapped mass ratio or a missing square root breaks the first."""
    rng = np.random.default_rng(3)
    mk, mj = rng.uniform(1e-5, 8e-5, 50), rng.uniform(1e-5, 8e-5, 50)
    Wk, Wj = rng.uniform(0.002, 0.05, 50), rng.uniform(0.002, 0.05, 50)
    lhs = TR.wilke_phi(mj, mk, Wj, Wk)
    rhs = (mj / mk) * (Wk / Wj) * TR.wilke_phi(mk, mj, Wk, Wj)
    assert np.allclose(lhs, rhs, rtol=1e-14, atol=0)
    assert np.allclose(TR.wilke_phi(mk, mk, Wk, Wk), 1.0, rtol=1e-15)


def test_binary_closed_forms():
    """Hand-derived values for two species of equal molar mass at equal mole
    fractions with mu_2 = 4 mu_1 and lam_2 = 4 lam_1: Phi_12 = 9/16,
    Phi_21 = 9/4, so mu = (16/25 + 16/13) mu_1 = 608/325 mu_1;
    lam = (5/2 + 8/5) lam_1 / 2 = 41/20 lam_1.  Binary diffusion:
    D_1m = D_12 W_2 / Wbar = D_12 y_2 / X_2."""
    W = np.array([0.028, 0.028])
    T = np.array([1000.0])
    p = np.array([101325.0])
    lnT = np.log(T[0])
    # constant fits: P_k = sqrt(mu_k) / T^(1/4), Q_k = lam_k / T^(1/2)
    mu1, lam1 = 2.0e-5, 0.03
    visc = np.zeros((2, 5))
    cond = np.zeros((2, 5))
    visc[0, 0] = np.sqrt(mu1) / T[0] ** 0.25
    visc[1, 0] = np.sqrt(4 * mu1) / T[0] ** 0.25
    cond[0, 0] = lam1 / np.sqrt(T[0])
    cond[1, 0] = 4 * lam1 / np.sqrt(T[0])
    diff = np.zeros((2, 2, 5))
    diff[0, 1, :2] = diff[1, 0, :2] = (1.0e-3, 2.0e-5)
    diff[0, 0, 0] = diff[1, 1, 0] = 5e-4
    mu, lam, D = TR.transport(visc, cond, diff, W, T, p, np.array([[0.5], [0.5]]))
    assert mu[0] == pytest.approx(608.0 / 325.0 * mu1, rel=1e-13)
    assert lam[0] == pytest.approx(41.0 / 20.0 * lam1, rel=1e-13)
    # unequal masses for the diffusion closed form
    W2 = np.array([0.002, 0.032])
    Y = np.array([[0.3], [0.7]])
    _, _, D = TR.transport(visc, cond, diff, W2, T, p, Y)
    D12 = T[0] ** 1.5 * (1.0e-3 + 2.0e-5 * lnT) / p[0]
    Wbar = 1.0 / (0.3 / 0.002 + 0.7 / 0.032)
    assert D[0, 0] == pytest.approx(D12 * W2[1] / Wbar, rel=1e-13)
    assert D[1, 0] == pytest.approx(D12 * W2[0] / Wbar, rel=1e-13)


def test_single_species_limits(m9fits):
    """A pure species: mu = mu_k, lam = lam_k (Wilke and Mathur reduce to the
    species' own values) and D_km = D_kk; negative and unnormalised inputs
    are clipped and normalised first."""
    m, (visc, cond, diff) = m9fits
    W = m.molar_masses()
    T = np.array([600.0, 1500.0, 2600.0])
    p = np.array([1e5, 2e5, 3e5])
    mu_k, lam_k = TR.pure_species(visc, cond, T)
    Db = TR.binary_diffusion(diff, T, p)
    for k in (0, 4, 8):
        Y = np.zeros((m.K, 3))
        Y[k] = [1.0, 2.0, 0.5]
        Y[(k + 1) % m.K] = -1e-9
        mu, lam, D = TR.transport(visc, cond, diff, W, T, p, Y)
        assert np.allclose(mu, mu_k[k], rtol=1e-14)
        assert np.allclose(lam, lam_k[k], rtol=1e-14)
        assert np.allclose(D[k], Db[k, k], rtol=1e-15)


def test_identical_species_split(m9fits):
    """Splitting one species into two copies of itself (same W, same fits)
    leaves mu, lam and every other species' D unchanged, at any split."""
    m, (visc, cond, diff) = m9fits
    W = m.molar_masses()
    K = m.K
    T, p, Y = _state(K, 40, 5)
    mu, lam, D = TR.transport(visc, cond, diff, W, T, p, Y)
    s = 2   # species split into s and K
    W2 = np.append(W, W[s])
    v2 = np.vstack([visc, visc[s]])
    c2 = np.vstack([cond, cond[s]])
    d2 = np.zeros((K + 1, K + 1, 5))
    d2[:K, :K] = diff
    d2[K, :K] = diff[s]
    d2[:K, K] = diff[:, s]
    d2[K, K] = diff[s, s]
    frac = np.random.default_rng(6).uniform(0, 1, 40)
    Y2 = np.vstack([Y, Y[s] * frac])
    Y2[s] *= 1 - frac
    mu2, lam2, D2 = TR.transport(v2, c2, d2, W2, T, p, Y2)
    assert np.allclose(mu2, mu, rtol=1e-13)
    assert np.allclose(lam2, lam, rtol=1e-13)
    keep = [k for k in range(K) if k != s]
    assert np.allclose(D2[keep], D[keep], rtol=1e-13)


def test_reordering_and_pressure(m9fits):
    """Permuting the species permutes D and leaves mu and lam; D scales as
    1/p while mu and lam do not depend on p."""
    m, (visc, cond, diff) = m9fits
    W = m.molar_masses()
    T, p, Y = _state(m.K, 30, 7)
    mu, lam, D = TR.transport(visc, cond, diff, W, T, p, Y)
    P = np.random.default_rng(8).permutation(m.K)
    mu2, lam2, D2 = TR.transport(visc[P], cond[P], diff[P][:, P], W[P], T, p, Y[P])
    assert np.allclose(mu2, mu, rtol=1e-13) and np.allclose(lam2, lam, rtol=1e-13)
    assert np.allclose(D2, D[P], rtol=1e-13)
    mu3, lam3, D3 = TR.transport(visc, cond, diff, W, T, 2.5 * p, Y)
    assert np.array_equal(mu3, mu) and np.array_equal(lam3, lam)
    assert np.allclose(D3 * 2.5, D, rtol=1e-14)


def test_fits_follow_kinetic_theory():
    """The seeded fits reproduce the Chapman-Enskog values they were made
    from within the fit error over 300-3500 K, and the properties are in the
    range of real gases (viscosity 2e-6 .. 3e-4 Pa s, binary diffusion
    1e-7 .. 5e-2 m^2/s at 1 atm)."""
    from chemgen import transport as CT
    m = standard_mechanism("M35")
    visc, cond, diff = transport_fits(m, 4)
    mu_k, lam_k = TR.pure_species(visc, cond, T_FIT)
    assert np.all((mu_k > 2e-6) & (mu_k < 3e-4)) and np.all(lam_k > 0)
    Db = TR.binary_diffusion(diff, T_FIT, np.full(T_FIT.size, 101325.0))
    assert np.all((Db > 1e-7) & (Db < 5e-2))
    assert np.allclose(Db, Db.transpose(1, 0, 2), rtol=0, atol=0)
    # viscosity of species 0 from its Lennard-Jones parameters, recomputed
    ref = CT.kinetic_viscosity(m, 4)
    assert np.allclose(mu_k, ref, rtol=5e-3)


def test_thermo_field_round_trip(om9):
    """T -> h(T, Y) -> T by the Newton from a guess 300 K away returns T, cp
    equals the temperature derivative of h, and an unreachable enthalpy
    gives NaN after 20 iterations."""
    m = standard_mechanism("M9")
    T, _, Y = _state(m.K, 25, 9, 450.0, 3000.0)
    h = np.array([om9.enthalpy(T[i], Y[:, i]) for i in range(25)])
    guess = np.where(T < 1800, T + 300.0, T - 300.0)
    T2, cp, its = TR.thermo_field(om9, h, Y, guess)
    assert np.allclose(T2, T, rtol=0, atol=1e-8)
    assert np.all((its >= 2) & (its <= 8))
    for i in range(0, 25, 6):
        d = 1e-3
        dh = (om9.enthalpy(T[i] + d, Y[:, i]) - om9.enthalpy(T[i] - d, Y[:, i])) / (2 * d)
        assert cp[i] == pytest.approx(dh, rel=1e-8)
    hb = np.array([h[0] + 1e9])
    Tb, cpb, itb = TR.thermo_field(om9, hb, Y[:, :1], np.array([1000.0]))
    assert np.isnan(Tb[0]) and np.isnan(cpb[0]) and itb[0] == 21
