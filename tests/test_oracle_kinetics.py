"""Pins of the oracle's thermo, kinetics, right-hand side and Jacobian.

Every check here is fixed by something other than the oracle's own formula:
closed forms of special cases, identities between thermo functions, conservation
invariants of the reactor equations, detailed balance at an equilibrium built
independently (from element potentials with the generator's own Gibbs
evaluation), complex-step and finite-difference derivatives, and a library
linear solver."""
import math

import numpy as np
import pytest

from chemgen.equilibrium import gibbs_over_RT
from chemgen.fields import cells4096, flame_field
from chemgen.mechanism import R_U, custom_mechanism, nasa_for, standard_mechanism

P = 101325.0


def _oracle_for(mech, tmp_path, oracle_lib, name="m.mech"):
    p = str(tmp_path / name)
    mech.write(p)
    return oracle_lib.OracleMech(p)


# --------------------------------------------------------------------------- thermo

def test_thermo_constant_cp_closed_form(tmp_path, oracle_lib):
    """cp/R = a1 constant: H/RT = a1 + a6/T, S/R = a1 ln T + a7."""
    coeffs = [[3.5, 0, 0, 0, 0, -1234.5, 6.75], [2.5, 0, 0, 0, 0, 2500.0, 4.0]]
    m = custom_mechanism([[1, 0], [0, 1]], coeffs, [([(0, 1)], [(1, 1)], 1e5, 0.0, 0.0)])
    om = _oracle_for(m, tmp_path, oracle_lib)
    for T in (250.0, 999.0, 1000.0, 2400.0, 3400.0):
        cp, h, s = om.thermo(T)
        for k, c in enumerate(coeffs):
            assert cp[k] == pytest.approx(c[0], rel=1e-15)
            assert h[k] == pytest.approx(c[0] + c[5] / T, rel=1e-14)
            assert s[k] == pytest.approx(c[0] * math.log(T) + c[6], rel=1e-14)


def test_thermo_formation_values(tmp_path, oracle_lib):
    """Coefficients built to give H(298.15) = dHf and S(298.15) = S0."""
    cps = [[3.0, 1e-3, -2e-7, 1e-11, -1e-15], [4.2, 2e-4, 0.0, 0.0, 0.0]]
    targets = [(-241.8e3, 188.8), (52.0e3, 219.3)]
    coeffs = [nasa_for(c, dh, s0) for c, (dh, s0) in zip(cps, targets)]
    m = custom_mechanism([[1, 0], [0, 1]], coeffs, [([(0, 1)], [(1, 1)], 1e5, 0.0, 0.0)])
    om = _oracle_for(m, tmp_path, oracle_lib)
    cp, h, s = om.thermo(298.15)
    for k, (dh, s0) in enumerate(targets):
        assert h[k] * R_U * 298.15 == pytest.approx(dh, rel=1e-12, abs=1e-6)
        assert s[k] * R_U == pytest.approx(s0, rel=1e-12)


def test_thermo_range_selection(tmp_path, oracle_lib):
    m = custom_mechanism([[1, 0], [0, 1]], [[3.0, 0, 0, 0, 0, 0, 0], [3.0, 0, 0, 0, 0, 0, 0]],
                         [([(0, 1)], [(1, 1)], 1e5, 0.0, 0.0)])
    m.nasa[0, 10:17] = [5.0, 0, 0, 0, 0, 0, 0]      # species 0: different high-range set
    om = _oracle_for(m, tmp_path, oracle_lib)
    assert om.thermo(999.9)[0][0] == 3.0
    assert om.thermo(1000.0)[0][0] == 5.0         # T < T_mid picks the low set


@pytest.mark.parametrize("T", [300.0, 800.0, 1500.0, 2500.0, 3300.0])
def test_thermo_derivative_identities(om35, T):
    """cp = dH/dT and dS/dT = cp/T, by 4th-order central differences."""
    d = 0.5

    def H(t):  # H/R
        return om35.thermo(t)[1] * t

    def S(t):
        return om35.thermo(t)[2]

    dH = (-H(T + 2 * d) + 8 * H(T + d) - 8 * H(T - d) + H(T - 2 * d)) / (12 * d)
    dS = (-S(T + 2 * d) + 8 * S(T + d) - 8 * S(T - d) + S(T - 2 * d)) / (12 * d)
    cp = om35.thermo(T)[0]
    assert np.allclose(dH, cp, rtol=1e-9)
    assert np.allclose(dS * T, cp, rtol=1e-9)


def test_gibbs_matches_independent_evaluation(om35, mech_dir):
    from chemgen.mechanism import read_mechanism
    m = read_mechanism(str(mech_dir / "M35.mech"))
    for T in (400.0, 1200.0, 2100.0):
        cp, h, s = om35.thermo(T)
        assert np.allclose(h - s, gibbs_over_RT(m.nasa, T), rtol=1e-13, atol=1e-11)


# --------------------------------------------------------------------------- rates

def test_arrhenius_units_and_activation(tmp_path, oracle_lib):
    """b = 0, Ea = 0: k_f equals A converted from cm-mol-s to SI; with Ea the
    ratio of rate constants at two temperatures is exp(-Ea/R (1/T1 - 1/T2))."""
    coeffs = [[3.5, 0, 0, 0, 0, 0, 0]] * 3
    rx = [([(0, 1), (1, 1)], [(2, 1)], 2.0e13, 0.0, 0.0),      # bimolecular: cm3/mol/s
          ([(2, 1)], [(0, 1), (1, 1)], 3.0e9, 0.0, 0.0),        # unimolecular: 1/s
          ([(0, 1), (1, 1)], [(2, 1)], 1.0e12, 0.0, 80e3),
          ([(0, 2)], [(1, 1)], 1.0e12, 0.7, 0.0)]
    m = custom_mechanism([[1, 0], [0, 1], [1, 1]], coeffs, rx)
    om = _oracle_for(m, tmp_path, oracle_lib)
    Y = np.array([0.3, 0.3, 0.4])
    kf1 = om.rates(1500.0, P, Y)[0]
    kf2 = om.rates(900.0, P, Y)[0]
    assert kf1[0] == pytest.approx(2.0e13 * 1e-6, rel=1e-15)
    assert kf1[1] == pytest.approx(3.0e9, rel=1e-15)
    assert kf1[2] / kf2[2] == pytest.approx(math.exp(-80e3 / R_U * (1 / 1500.0 - 1 / 900.0)), rel=1e-13)
    assert kf1[3] / kf2[3] == pytest.approx((1500.0 / 900.0) ** 0.7, rel=1e-14)


@pytest.mark.parametrize("T", [500.0, 1100.0, 2000.0])
def test_reverse_rate_is_equilibrium_constant(om9, mech_dir, T):
    """k_f / k_r = K_c = exp(-sum nu g) (p0/RT)^dnu with g from the generator's
    own (independent) Gibbs evaluation."""
    from chemgen.mechanism import read_mechanism
    m = read_mechanism(str(mech_dir / "M9.mech"))
    g = gibbs_over_RT(m.nasa, T)
    Y = np.full(m.K, 1.0 / m.K)
    kf, kr, q, wd = om9.rates(T, P, Y)
    for i, (reac, prod, *_ ) in enumerate(m.reactions):
        dnu = sum(nu for _, nu in prod) - sum(nu for _, nu in reac)
        dg = sum(nu * g[k] for k, nu in prod) - sum(nu * g[k] for k, nu in reac)
        Kc = math.exp(-dg) * (P / (R_U * T)) ** dnu
        assert kf[i] / kr[i] == pytest.approx(Kc, rel=1e-11)


def _equilibrium_state(m, T, rng):
    """X_k = exp(-g_k + n_k . lam) for random element potentials, shifted so that
    sum X = 1 (monotone in the shift since every species has >= 1 atom)."""
    n = m.counts.astype(float)
    g = gibbs_over_RT(m.nasa, T)
    lam = rng.uniform(-5, 5, size=m.E) + np.min(g / n.sum(1))
    atoms = n.sum(1)
    lo, hi = -200.0, 200.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        u = -g + n @ lam + mid * atoms
        s = np.exp(np.minimum(u, 700)).sum()
        lo, hi = (lo, mid) if s > 1 else (mid, hi)
    X = np.exp(-g + n @ lam + 0.5 * (lo + hi) * atoms)
    X /= X.sum()
    W = m.molar_masses()
    Y = X * W / (X * W).sum()
    return Y


@pytest.mark.parametrize("T", [700.0, 1500.0, 2300.0])
def test_detailed_balance_at_equilibrium(om9, mech_dir, T):
    from chemgen.mechanism import read_mechanism
    m = read_mechanism(str(mech_dir / "M9.mech"))
    rng = np.random.default_rng(int(T))
    for _ in range(5):
        Y = _equilibrium_state(m, T, rng)
        kf, kr, q, wd = om9.rates(T, P, Y)
        W = m.molar_masses()
        rho = P / (R_U * T) / np.sum(Y / W)
        C = rho * Y / W
        for i, (reac, prod, *_ ) in enumerate(m.reactions):
            fwd = kf[i] * np.prod([C[k] ** nu for k, nu in reac])
            rev = kr[i] * np.prod([C[k] ** nu for k, nu in prod])
            scale = max(fwd, rev)
            if scale > 1e-250:
                assert abs(q[i]) <= 1e-11 * scale


# --------------------------------------------------------------------------- RHS

def _states(m, n=24, seed=5):
    f = cells4096(m, n=n, seed=seed)
    return [np.append(f.Y[:, i], f.T[i]) for i in range(n)]


@pytest.mark.parametrize("which", ["M9", "M35"])
def test_rhs_conservation_invariants(which, om9, om35, mech_dir):
    from chemgen.mechanism import read_mechanism
    om = om9 if which == "M9" else om35
    m = read_mechanism(str(mech_dir / f"{which}.mech"))
    W = m.molar_masses()
    for y in _states(m):
        Y, T = y[:-1], y[-1]
        kf, kr, q, wd = om.rates(T, P, Y)
        f = om.rhs(P, y)
        # total mass: sum_k W_k wdot_k = 0
        terms = np.concatenate([[W[k] * nu * q[i] for k, nu in r] + [W[k] * nu * q[i] for k, nu in pr]
                                for i, (r, pr, *_ ) in enumerate(m.reactions)])
        assert abs(np.sum(W * wd)) <= 1e-14 * np.abs(terms).sum()
        assert abs(np.sum(f[:-1])) <= 1e-14 * np.abs(f[:-1]).sum() + 1e-300
        # element conservation: sum_k n_ke wdot_k = 0
        for e in range(m.E):
            tot = m.counts[:, e] @ wd
            assert abs(tot) <= 1e-13 * (np.abs(m.counts[:, e]) @ np.abs(wd)) + 1e-300
        # enthalpy: dh/dt = sum_k h_k dY_k/dt + cp dT/dt = 0
        cp_R, h_RT, s_R = om.thermo(T)
        hk = h_RT * R_U * T / W
        cpm = np.sum(Y * cp_R * R_U / W)
        dh = hk @ f[:-1] + cpm * f[-1]
        assert abs(dh) <= 1e-12 * np.abs(hk * f[:-1]).sum()


def test_rhs_equilibrium_is_stationary(om9, mech_dir):
    from chemgen.mechanism import read_mechanism
    m = read_mechanism(str(mech_dir / "M9.mech"))
    Y = _equilibrium_state(m, 1800.0, np.random.default_rng(3))
    f = om9.rhs(P, np.append(Y, 1800.0))
    kf, kr, q, wd = om9.rates(1800.0, P, Y)
    assert np.all(np.abs(f[:-1]) <= 1e-10 * (np.abs(kf).max() + 1.0))


# --------------------------------------------------------------------------- Jacobian

@pytest.mark.parametrize("which", ["M9", "M35"])
def test_jacobian_vs_complex_step(which, om9, om35, mech_dir):
    from chemgen.mechanism import read_mechanism
    om = om9 if which == "M9" else om35
    m = read_mechanism(str(mech_dir / f"{which}.mech"))
    for y in _states(m, n=8):
        J = om.jac(P, y)
        Jc = om.jac_cs(P, y)
        scale = np.abs(Jc).max(axis=1, keepdims=True) + 1e-300
        assert np.max(np.abs(J - Jc) / scale) <= 1e-12


def test_jacobian_vs_finite_difference(om9, mech_dir):
    from chemgen.mechanism import read_mechanism
    m = read_mechanism(str(mech_dir / "M9.mech"))
    y = _states(m, n=1, seed=11)[0]
    J = om9.jac(P, y)
    N = y.size
    Jfd = np.zeros((N, N))
    for j in range(N):
        d = 1e-6 * max(abs(y[j]), 1e-3)
        yp, ym = y.copy(), y.copy()
        yp[j] += d
        ym[j] -= d
        Jfd[:, j] = (om9.rhs(P, yp) - om9.rhs(P, ym)) / (2 * d)
    scale = np.abs(J).max(axis=1, keepdims=True)
    assert np.max(np.abs(J - Jfd) / scale) <= 1e-5


# --------------------------------------------------------------------------- T from h

def test_T_newton_roundtrip(om35, mech_dir):
    from chemgen.mechanism import read_mechanism
    m = read_mechanism(str(mech_dir / "M35.mech"))
    f = cells4096(m, n=16, seed=9)
    for i in range(16):
        Y = f.Y[:, i]
        for T in (250.0, 600.0, 1400.0, 2300.0, 3000.0):
            h0 = om35.enthalpy(T, Y)
            T2, it = om35.T_from_h(h0, Y, T + 150.0 if T < 2900 else T - 150.0)
            assert abs(T2 - T) <= 1e-10
            assert it <= 20


# --------------------------------------------------------------------------- LU

def test_lu_matches_library_solver(oracle_lib):
    rng = np.random.default_rng(0)
    for N in (1, 2, 10, 36):
        A = rng.standard_normal((N, N)) * 10.0 ** rng.uniform(-3, 3, size=(N, 1))
        b = rng.standard_normal(N)
        LU, piv, bad = oracle_lib.lu(A)
        assert bad == 0
        x = oracle_lib.lu_solve(LU, piv, b)
        assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-9, atol=1e-12)


def test_lu_pivot_ties_and_singular(oracle_lib):
    A = np.array([[1.0, 2.0], [-1.0, 3.0]])       # |a00| == |a10|: keep row 0
    LU, piv, bad = oracle_lib.lu(A)
    assert piv[0] == 0 and bad == 0
    A = np.array([[1.0, 2.0], [-2.0, 3.0]])
    LU, piv, bad = oracle_lib.lu(A)
    assert piv[0] == 1
    _, _, bad = oracle_lib.lu(np.array([[0.0, 1.0], [0.0, 2.0]]))
    assert bad == 1
