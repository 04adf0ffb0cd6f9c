"""Pins of the oracle's real-mechanism kinetics (third-body efficiencies,
Lindemann and Troe fall-off, duplicate and irreversible reactions, two NASA-7
ranges), each against something other than the oracle's own formula: limits
of the fall-off blend, the Troe form at the centre of its broadening curve,
special cases that reduce to another form, ideal-gas totals, equilibrium
states from the element-potential solver of the input generator, and the
complex-step derivative of the right-hand side.

The paper runs an H2 mechanism (9 species, Section 4.1) and a CH4 mechanism
(20 species, Section 4.2); those files are not available, so the seeded
stand-ins H2R and CH4R carry the same kinds of reactions at the same sizes."""
import dataclasses
import math

import numpy as np
import pytest

from chemgen.equilibrium import element_moles, equilibrium_mass_fractions, gibbs_over_RT
from chemgen.mechanism import (R_U, REAL_LIKE_SPECS, RxnKinetics, custom_mechanism, read_mechanism,
                               standard_mechanism)

P = 101325.0
LN10 = math.log(10.0)


def _om(mech, tmp_path, oracle_lib, name="m.mech"):
    p = str(tmp_path / name)
    mech.write(p)
    return oracle_lib.OracleMech(p)


def _arrh(A_si, b, Ea, T):
    return A_si * T ** b * math.exp(-Ea / (R_U * T))


# A + B (+M) <=> AB (+M) among three species of two elements, constant cp
COUNTS = [[1, 0], [0, 1], [1, 1]]
COEFFS = [[3.5, 0, 0, 0, 0, -1000.0, 4.0], [3.5, 0, 0, 0, 0, -2000.0, 5.0], [4.5, 0, 0, 0, 0, -30000.0, 3.0]]
RX = [([(0, 1), (1, 1)], [(2, 1)], 2.0e13, 0.3, 20e3)]


def _one(kind, tmp_path, oracle_lib, **kw):
    x = RxnKinetics(kind=kind, **kw)
    return _om(custom_mechanism(COUNTS, COEFFS, RX, kinetics=[x]), tmp_path, oracle_lib, f"{kind}.mech")


# --------------------------------------------------------------------------- generator

@pytest.mark.parametrize("name", sorted(REAL_LIKE_SPECS))
def test_real_like_mechanisms(name, tmp_path):
    """Sizes and feature counts as specified; every species has a second NASA
    range that differs from the first but meets it at Tmid in cp, H and S;
    the version 2 text reads back to the same mechanism."""
    spec = REAL_LIKE_SPECS[name]
    m = standard_mechanism(name)
    assert (m.K, m.R) == (spec["K"], spec["R"])
    kinds = [m.kin(i).kind for i in range(m.R)]
    dups = m.R - len({(tuple(r), tuple(p)) for r, p, *_ in m.reactions})
    assert dups == spec["n_dup"]
    assert kinds.count("third") >= spec["n_third"]
    assert kinds.count("lind") >= spec["n_lind"]
    assert kinds.count("troe3") + kinds.count("troe4") >= spec["n_troe"]
    assert sum(not m.kin(i).reversible for i in range(m.R)) >= spec["n_irrev"]
    assert any(m.kin(i).default_eff == 0.0 for i in range(m.R))
    for k in range(m.K):
        lo, hi, tm = m.nasa[k, 3:10], m.nasa[k, 10:17], m.nasa[k, 1]
        assert not np.allclose(lo, hi)
        cp = [np.polyval(a[4::-1], tm) for a in (lo, hi)]
        h = [np.polyval((a[:5] / np.arange(1, 6))[::-1], tm) * tm + a[5] for a in (lo, hi)]
        s = [a[0] * math.log(tm) + np.polyval((a[1:5] / np.arange(1, 5))[::-1], tm) * tm + a[6] for a in (lo, hi)]
        assert cp[0] == pytest.approx(cp[1], rel=1e-12)
        assert h[0] == pytest.approx(h[1], rel=1e-9, abs=1e-6)
        assert s[0] == pytest.approx(s[1], rel=1e-12)
    path = str(tmp_path / f"{name}.mech")
    m.write(path)
    assert open(path).readline().split() == ["CHEMMECH", "2"]
    back = read_mechanism(path)
    assert back.to_text() == m.to_text()


def test_plain_mechanisms_keep_format_1(tmp_path):
    p = str(tmp_path / "m9.mech")
    standard_mechanism("M9").write(p)
    assert open(p).readline().split() == ["CHEMMECH", "1"]


# --------------------------------------------------------------------------- thermo

@pytest.mark.parametrize("name", sorted(REAL_LIKE_SPECS))
def test_two_range_thermo(name, tmp_path, oracle_lib):
    """Above Tmid the oracle uses the high range: H is continuous across Tmid,
    dH/dT = cp on both sides (central differences), and above Tmid H differs
    from the low range carried past Tmid."""
    m = standard_mechanism(name)
    om = _om(m, tmp_path, oracle_lib)
    tm = m.nasa[0, 1]
    cpa, ha, _ = om.thermo(tm * (1 - 1e-12))
    cpb, hb, _ = om.thermo(tm)
    assert np.allclose(ha * tm * (1 - 1e-12), hb * tm, rtol=1e-9, atol=1e-6)
    for T in (tm - 300.0, tm + 700.0):
        d = 1e-3
        cp, _, _ = om.thermo(T)
        hp = om.thermo(T + d)[1] * (T + d)
        hm = om.thermo(T - d)[1] * (T - d)
        assert np.allclose((hp - hm) / (2 * d), cp, rtol=1e-7)
    T = tm + 1500.0
    lo = m.nasa[:, 3:10]
    h_lo = lo[:, 0] + lo[:, 1] * T / 2 + lo[:, 2] * T ** 2 / 3 + lo[:, 3] * T ** 3 / 4 + lo[:, 4] * T ** 4 / 5 + lo[:, 5] / T
    assert np.all(np.abs(om.thermo(T)[1] - h_lo) > 1e-6)


# --------------------------------------------------------------------------- rate forms

def test_third_body_is_total_concentration(tmp_path, oracle_lib):
    """Efficiencies 1: [M] is the ideal-gas total p/(RT), so k_f = k p/(RT)
    with A converted from cm^6/mol^2/s; a species of efficiency 0 that is the
    only one present gives k_f = 0; a single bath species (default 0) gives
    [M] = its concentration."""
    T = 1300.0
    om = _one("third", tmp_path, oracle_lib)
    k = _arrh(2.0e13 * 1e-12, 0.3, 20e3, T)
    for Y in ([0.2, 0.3, 0.5], [1.0, 0.0, 0.0]):
        kf = om.rates(T, P, np.array(Y))[0][0]
        assert kf == pytest.approx(k * P / (R_U * T), rel=1e-13)
    om0 = _one("third", tmp_path, oracle_lib, effs=[(2, 0.0)])
    assert om0.rates(T, P, np.array([0.0, 0.0, 1.0]))[0][0] == 0.0
    omb = _one("third", tmp_path, oracle_lib, default_eff=0.0, effs=[(1, 1.0)])
    assert omb.rates(T, P, np.array([0.0, 1.0, 0.0]))[0][0] == pytest.approx(k * P / (R_U * T), rel=1e-13)
    assert omb.rates(T, P, np.array([0.5, 0.0, 0.5]))[0][0] == 0.0


def test_falloff_limits(tmp_path, oracle_lib):
    """Lindemann: k_f -> k_inf at high [M] and k_f -> k_0 [M] at low [M]
    (relative deviations of order 1/Pr and Pr)."""
    T = 1500.0
    low = (3.0e18, -1.2, 4000.0)
    om = _one("lind", tmp_path, oracle_lib, low=low)
    kinf = _arrh(2.0e13 * 1e-6, 0.3, 20e3, T)
    k0 = _arrh(low[0] * 1e-12, low[1], low[2], T)
    Y = np.array([0.2, 0.3, 0.5])
    for p in (1e16, 1e18):
        M = p / (R_U * T)
        Pr = k0 * M / kinf
        assert Pr > 1e5
        assert om.rates(T, p, Y)[0][0] == pytest.approx(kinf, rel=2.0 / Pr)
    for p in (1e-5, 1e-7):
        M = p / (R_U * T)
        Pr = k0 * M / kinf
        assert Pr < 1e-5
        assert om.rates(T, p, Y)[0][0] == pytest.approx(k0 * M, rel=2.0 * Pr)


@pytest.mark.parametrize("kind,troe", [("troe3", (0.62, 180.0, 1900.0)), ("troe4", (0.41, 95.0, 2600.0, 5100.0))])
@pytest.mark.parametrize("T", [600.0, 1400.0, 2500.0])
def test_troe_centre_of_broadening(kind, troe, T, tmp_path, oracle_lib):
    """At log10 Pr = 0.4 + 0.67 log10 Fcent (the centre of the broadening
    curve, f = 0) the Troe factor equals Fcent, whose closed form is
    (1 - a) exp(-T/T3) + a exp(-T/T1) [+ exp(-T2/T)]."""
    low = (3.0e18, -1.2, 4000.0)
    om = _one(kind, tmp_path, oracle_lib, low=low, troe=troe)
    a, T3, T1 = troe[:3]
    Fc = (1 - a) * math.exp(-T / T3) + a * math.exp(-T / T1) + (math.exp(-troe[3] / T) if len(troe) == 4 else 0.0)
    Pr = 10.0 ** (0.4 + 0.67 * math.log10(Fc))
    kinf = _arrh(2.0e13 * 1e-6, 0.3, 20e3, T)
    k0 = _arrh(low[0] * 1e-12, low[1], low[2], T)
    p = Pr * kinf / k0 * R_U * T          # [M] = p/(RT) with unit efficiencies
    kf = om.rates(T, p, np.array([0.2, 0.3, 0.5]))[0][0]
    assert kf / (kinf * Pr / (1 + Pr)) == pytest.approx(Fc, rel=1e-11)


@pytest.mark.parametrize("T", [900.0, 1700.0, 2600.0])
def test_troe_factor_is_one_at_its_pole(T, tmp_path, oracle_lib):
    """The Troe argument f = u / (n - 0.14 u), u = log10 Pr + c, has a pole at
    u = n / 0.14, where the broadening factor is exactly 1 (k_f equals the
    Lindemann value); this fixes the width constant 0.14, which the centre
    of the curve does not see."""
    troe, low = (0.45, 120.0, 2200.0), (3.0e18, -1.2, 4000.0)
    om = _one("troe3", tmp_path, oracle_lib, low=low, troe=troe)
    Fc = (1 - troe[0]) * math.exp(-T / troe[1]) + troe[0] * math.exp(-T / troe[2])
    Lc = math.log10(Fc)
    c, n = -0.4 - 0.67 * Lc, 0.75 - 1.27 * Lc
    Pr = 10.0 ** (n / 0.14 - c)
    kinf = _arrh(2.0e13 * 1e-6, 0.3, 20e3, T)
    k0 = _arrh(low[0] * 1e-12, low[1], low[2], T)
    p = Pr * kinf / k0 * R_U * T
    kf = om.rates(T, p, np.array([0.2, 0.3, 0.5]))[0][0]
    assert kf == pytest.approx(kinf * Pr / (1 + Pr), rel=1e-9)
    # away from the pole the factor is below 1
    assert om.rates(T, 0.5 * p, np.array([0.2, 0.3, 0.5]))[0][0] < 0.5 * kinf * Pr / (1 + 0.5 * Pr) * (1 - 1e-6)


def test_troe_with_unit_fcent_is_lindemann(tmp_path, oracle_lib):
    """a = 0 and T3 huge make Fcent = 1, and the Troe form reduces to Lindemann
    at every pressure; with Fcent < 1 the Troe factor lies in (0, 1]."""
    low = (3.0e18, -1.2, 4000.0)
    oml = _one("lind", tmp_path, oracle_lib, low=low)
    omt = _one("troe3", tmp_path, oracle_lib, low=low, troe=(0.0, 1e300, 1000.0))
    omr = _one("troe3", tmp_path, oracle_lib, low=low, troe=(0.6, 200.0, 1500.0))
    Y = np.array([0.2, 0.3, 0.5])
    for T in (800.0, 1800.0):
        for p in 10.0 ** np.arange(-2.0, 12.0, 1.0):
            kl, kt, kr = oml.rates(T, p, Y)[0][0], omt.rates(T, p, Y)[0][0], omr.rates(T, p, Y)[0][0]
            assert kt == pytest.approx(kl, rel=1e-14)
            assert 0.0 < kr <= kl * (1 + 1e-14)


def test_duplicates_add_and_irreversible_has_no_reverse(tmp_path, oracle_lib):
    """Two duplicate reactions with pre-exponentials A1 and A2 (same b, Ea)
    give the right-hand side of one reaction with A1 + A2; an irreversible
    reaction has k_r = 0 and q = k_f prod C."""
    rx2 = [RX[0], (RX[0][0], RX[0][1], 5.0e12, 0.3, 20e3)]
    m2 = custom_mechanism(COUNTS, COEFFS, rx2)
    m1 = custom_mechanism(COUNTS, COEFFS, [(RX[0][0], RX[0][1], 2.5e13, 0.3, 20e3)])
    om2, om1 = _om(m2, tmp_path, oracle_lib, "d2.mech"), _om(m1, tmp_path, oracle_lib, "d1.mech")
    y = np.array([0.2, 0.3, 0.5, 1700.0])
    assert np.allclose(om2.rhs(P, y), om1.rhs(P, y), rtol=1e-14, atol=0)
    omi = _one("elem", tmp_path, oracle_lib, reversible=False)
    kf, kr, q, wd = omi.rates(1700.0, P, y[:3])
    W = custom_mechanism(COUNTS, COEFFS, RX).molar_masses()
    rho = P / (R_U * 1700.0) / np.sum(y[:3] / W)
    C = rho * y[:3] / W
    assert kr[0] == 0.0 and q[0] == pytest.approx(kf[0] * C[0] * C[1], rel=1e-14)


# --------------------------------------------------------------------------- balance and Jacobian

@pytest.mark.parametrize("name", sorted(REAL_LIKE_SPECS))
def test_pressure_dependent_detailed_balance(name, tmp_path, oracle_lib):
    """Detailed balance with pressure-dependent rates: at chemical equilibrium
    (element-potential solver of the input generator, its own Gibbs
    evaluation) every reversible reaction's rate of progress vanishes at any
    pressure, and k_f / k_r = K_c(T) does not depend on the pressure."""
    m = standard_mechanism(name)
    om = _om(m, tmp_path, oracle_lib)
    W = m.molar_masses()
    rng = np.random.default_rng(3)
    for T in (900.0, 1600.0, 2400.0):
        g = gibbs_over_RT(m.nasa, T)
        Kc = []
        for p in (1e3, P, 3e6):
            Y0 = rng.dirichlet(np.ones(m.K))
            Y = equilibrium_mass_fractions(m, T, p, element_moles(m, Y0))
            kf, kr, q, wd = om.rates(T, p, Y)
            rho = p / (R_U * T) / np.sum(Y / W)
            C = rho * Y / W
            Kc.append([kf[i] / kr[i] if m.kin(i).reversible else 0.0 for i in range(m.R)])
            for i, (reac, prod, *_ ) in enumerate(m.reactions):
                if not m.kin(i).reversible:
                    assert kr[i] == 0.0
                    continue
                fwd = kf[i] * np.prod([C[k] ** nu for k, nu in reac])
                if fwd > 1e-250:
                    assert abs(q[i]) <= 1e-8 * fwd, (name, T, p, i)
                dnu = sum(nu for _, nu in prod) - sum(nu for _, nu in reac)
                dg = sum(nu * g[k] for k, nu in prod) - sum(nu * g[k] for k, nu in reac)
                assert kf[i] / kr[i] == pytest.approx(math.exp(-dg) * (P / (R_U * T)) ** dnu, rel=1e-10)
        assert np.allclose(Kc[0], Kc[1], rtol=1e-12) and np.allclose(Kc[0], Kc[2], rtol=1e-12)


@pytest.mark.parametrize("name", sorted(REAL_LIKE_SPECS))
def test_jacobian_matches_complex_step(name, tmp_path, oracle_lib):
    """The analytic Jacobian (fall-off derivatives in T and through [M]
    included) equals the complex-step derivative of the right-hand side over
    states from near-vacuum to high pressure, both sides of Tmid."""
    m = standard_mechanism(name)
    om = _om(m, tmp_path, oracle_lib)
    rng = np.random.default_rng(11)
    for _ in range(24):
        Y = rng.dirichlet(np.full(m.K, 0.5))
        T = rng.uniform(400.0, 2900.0)
        p = 10.0 ** rng.uniform(2.0, 7.5)
        y = np.append(Y, T)
        J, Jc = om.jac(p, y), om.jac_cs(p, y)
        scale = np.abs(Jc).max(axis=1, keepdims=True) + 1e-300
        assert np.max(np.abs(J - Jc) / scale) < 1e-10


def test_rejects_bad_kinetics(tmp_path, oracle_lib):
    """Damaged version 2 tails are rejected (unknown kind, efficiency of an
    unknown species, negative efficiency, missing Troe parameters)."""
    good = custom_mechanism(COUNTS, COEFFS, RX, kinetics=[RxnKinetics(kind="troe3", low=(1e18, 0, 0),
                                                                      troe=(0.5, 100.0, 1000.0), effs=[(1, 2.0)])])
    p = str(tmp_path / "g.mech")
    good.write(p)
    oracle_lib.OracleMech(p)
    text = open(p).read()
    line = [ln for ln in text.splitlines() if ln.startswith("R0 ")][0]
    for bad in (line.replace(" troe3 ", " troe9 "), line.replace(" 1 2.0", " 7 2.0"),
                line.replace(" 1 2.0", " 1 -2.0"), line.rsplit(" ", 6)[0]):
        q = tmp_path / "b.mech"
        q.write_text(text.replace(line, bad))
        with pytest.raises(Exception):
            oracle_lib.OracleMech(str(q))
