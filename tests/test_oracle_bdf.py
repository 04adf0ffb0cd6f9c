"""Pins of the oracle's BDF integrator.

* coefficients: the constant-step Nordsieck BDF vectors of the literature;
* exactness: variable-step BDF of order q reproduces polynomial solutions of
  degree <= q (and not degree q+1);
* observed order on the Prothero-Robinson problem;
* closed forms: A <-> B isomerisation relaxes exponentially; with unequal
  enthalpies, T follows from enthalpy conservation and the system reduces to a
  scalar ODE solved here independently;
* brute force: classical RK4 with step halving on a mild mechanism;
* invariants: element mass and enthalpy conservation, tolerance-sweep
  convergence; failure statuses restore the input state.
"""
import math

import numpy as np
import pytest

from chemgen.fields import cells4096, flame_field
from chemgen.mechanism import R_U, custom_mechanism, make_mechanism, standard_mechanism

P = 101325.0


def _oracle_for(mech, tmp_path, oracle_lib, name="m.mech"):
    p = str(tmp_path / name)
    mech.write(p)
    return oracle_lib.OracleMech(p)


# --------------------------------------------------------------------------- coefficients

def test_constant_step_coefficients(oracle_lib):
    # Nordsieck-form BDF vectors l (l0 = 1) for equal steps, orders 1..5
    ref = {1: [1, 1], 2: [1, 3 / 2, 1 / 2], 3: [1, 11 / 6, 1, 1 / 6],
           4: [1, 25 / 12, 35 / 24, 5 / 12, 1 / 24],
           5: [1, 137 / 60, 15 / 8, 17 / 24, 1 / 8, 1 / 120]}
    for q, l_ref in ref.items():
        xi, l = oracle_lib.bdf_coeffs(q, 0.1, [0.0] + [0.1] * 6)
        assert np.allclose(l, l_ref, rtol=1e-14)
        assert np.allclose(xi, np.arange(1, q + 2), rtol=1e-14)


def test_variable_step_coefficients_interpolate(oracle_lib):
    """Lambda(x) = sum l_j x^j vanishes at the past nodes x = -xi_i and is 1 at 0."""
    h, tau = 0.3, [0.0, 0.2, 0.5, 0.11, 0.7, 0.05]
    for q in range(1, 6):
        xi, l = oracle_lib.bdf_coeffs(q, h, tau)
        t_past = np.cumsum([h] + tau[1:q + 1])
        assert np.allclose(xi, t_past / h)
        for i in range(q):
            assert abs(np.polyval(l[::-1], -xi[i])) < 1e-12


# --------------------------------------------------------------------------- exactness

def _poly_problem(coef, lam):
    """y' = lam (y - p(t)) + p'(t): solution p(t) when y(0) = p(0)."""
    pc = np.array(coef, dtype=float)          # ascending powers
    dpc = np.array([k * pc[k] for k in range(1, len(pc))] or [0.0])

    def p(t):
        return np.polyval(pc[::-1], t)

    def dp(t):
        return np.polyval(dpc[::-1], t)

    f = lambda t, y: np.array([lam * (y[0] - p(t)) + dp(t)])
    j = lambda t, y: np.array([[lam]])
    return p, f, j, pc


def _nordsieck_of_poly(pc, t0, h, q):
    z = np.zeros((q + 1, 1))
    for jdx in range(q + 1):
        d = np.polyder(np.poly1d(pc[::-1]), jdx) if jdx else np.poly1d(pc[::-1])
        z[jdx, 0] = d(t0) * h ** jdx / math.factorial(jdx)
    return z


@pytest.mark.parametrize("q", [1, 2, 3, 4, 5])
def test_exact_on_polynomials_with_variable_steps(oracle_lib, q):
    rng = np.random.default_rng(q)
    coef = rng.uniform(-1, 1, size=q + 1)
    p, f, j, pc = _poly_problem(coef, lam=-50.0)
    hseq = rng.uniform(0.02, 0.08, size=12)
    t0 = 0.3
    z0 = _nordsieck_of_poly(pc, t0, hseq[0], q)
    tau = [0.0] + list(rng.uniform(0.02, 0.08, size=q + 1))
    z, _, bad = oracle_lib.bdf_prescribed(f, j, q, t0, z0, tau, hseq)
    assert bad == 0
    t_end = t0 + hseq.sum()
    assert abs(z[0, 0] - p(t_end)) <= 1e-12 * (1 + abs(p(t_end)))
    # degree q+1 is not reproduced: the test can tell
    coef2 = np.append(coef, 1.0)
    p2, f2, j2, pc2 = _poly_problem(coef2, lam=-50.0)
    z2, _, _ = oracle_lib.bdf_prescribed(f2, j2, q, t0, _nordsieck_of_poly(pc2, t0, hseq[0], q), tau, hseq)
    assert abs(z2[0, 0] - p2(t_end)) > 1e-9


@pytest.mark.parametrize("q", [1, 2, 3, 4, 5])
def test_observed_order_prothero_robinson(oracle_lib, q):
    lam = -10.0
    f = lambda t, y: np.array([lam * (y[0] - math.sin(t)) + math.cos(t)])
    j = lambda t, y: np.array([[lam]])
    errs = []
    for nsteps in (40, 80, 160):
        h = 1.0 / nsteps
        z0 = np.array([[math.sin(0.0) if k % 4 == 0 else (math.cos(0.0) if k % 4 == 1 else
                        (-math.sin(0.0) if k % 4 == 2 else -math.cos(0.0)))] for k in range(q + 1)])
        z0 = np.array([[z0[k, 0] * h ** k / math.factorial(k)] for k in range(q + 1)])
        tau = [0.0] + [h] * 6
        z, _, _ = oracle_lib.bdf_prescribed(f, j, q, 0.0, z0, tau, [h] * nsteps)
        errs.append(abs(z[0, 0] - math.sin(1.0)))
    for a, b in zip(errs, errs[1:]):
        order = math.log2(a / b)
        assert q - 0.3 <= order <= q + 0.6, (q, errs)


# --------------------------------------------------------------------------- closed forms

def _isomer_mech(kf_plus_kr, K_eq, dh=0.0):
    """A <-> B isomers (same element counts: identical molar mass) padded with 7
    inert species to 9.  Both species have cp/R = 3.5.  a7_B - a7_A = ln K so that
    K_c = K at any T when dh = 0."""
    k_f = kf_plus_kr * K_eq / (1.0 + K_eq)
    cA = [3.5, 0, 0, 0, 0, 0.0, 10.0]
    cB = [3.5, 0, 0, 0, 0, -dh / R_U, 10.0 + math.log(K_eq)]
    counts = [[1, 1], [1, 1]] + [[1, 0]] * 4 + [[0, 1]] * 3
    coeffs = [cA, cB] + [[3.0, 0, 0, 0, 0, 0.0, 5.0]] * 7
    return custom_mechanism(counts, coeffs, [([(0, 1)], [(1, 1)], k_f, 0.0, 0.0)])


@pytest.mark.parametrize("rate", [1e3, 1e6, 1e9, 1e12])
def test_isomerisation_closed_form(tmp_path, oracle_lib, rate):
    K_eq = 2.5
    m = _isomer_mech(rate, K_eq)
    om = _oracle_for(m, tmp_path, oracle_lib)
    n = 6
    Y = np.zeros((9, n))
    rng = np.random.default_rng(1)
    Y[0] = rng.uniform(0.05, 0.6, n)
    Y[1] = rng.uniform(0.0, 0.3, n)
    Y[2] = 1.0 - Y[0] - Y[1]
    T = rng.uniform(600, 2000, n)
    dt = 3.0 / rate
    errs = []
    for rtol in (1e-6, 1e-8, 1e-10):
        T1, Y1, st, cnt, _ = om.integrate(T, np.full(n, P), Y, dt, rtol=rtol, atol=1e-12 * rtol / 1e-8)
        assert np.all(st == 0)
        Yeq = (Y[0] + Y[1]) / (1.0 + K_eq)
        exact = Yeq + (Y[0] - Yeq) * math.exp(-rate * dt)
        err = np.abs(Y1[0] - exact)
        # global error: the WRMS local tolerance over N = 10 components allows
        # ~sqrt(10) per component, and local errors accumulate over ~100 steps
        assert np.all(err <= 100 * (rtol * np.abs(exact) + 1e-12))
        errs.append(err.max())
        assert np.allclose(T1, T, rtol=1e-12)
    assert errs[0] > 30 * errs[1] and errs[1] > 30 * errs[2]     # tolerance proportional


def test_isomerisation_with_heat_release(tmp_path, oracle_lib):
    """Unequal enthalpies: h is conserved, so with constant cp T is an explicit
    function of Y_B and dY_B/dt = r(Y_B) is a scalar ODE, integrated here by
    RK4 with step halving (independent of the oracle)."""
    K0, dh = 3.0, -40e3
    m = _isomer_mech(1.0, K0, dh=dh)
    # Arrhenius forward rate with activation energy: exercises k_f(T) and K_c(T)
    A, Ea = 2e7, 60e3
    m.reactions[0] = ([(0, 1)], [(1, 1)], A, 0.0, Ea)
    om = _oracle_for(m, tmp_path, oracle_lib)
    W = m.molar_masses()
    yA0, yB0, T0 = 0.2, 0.4, 1200.0
    Y = np.zeros(9)
    Y[0], Y[1], Y[2] = yA0, yB0, 1 - yA0 - yB0
    cpm = sum(Y[k] * m.nasa[k, 3] * R_U / W[k] for k in range(9))      # constant in time

    def T_of(yB):   # h = sum Y_k (cp_k T + H0_k)/W_k is conserved; H_B - H_A = -dh
        return T0 - (yB - yB0) * (-dh) / W[0] / cpm

    def r(yB):
        T = T_of(yB)
        yA = yA0 + yB0 - yB
        kf = A * math.exp(-Ea / (R_U * T))
        gA = 3.5 + 0.0 / T - 3.5 * math.log(T) - 10.0
        gB = 3.5 + (-dh / R_U) / T - 3.5 * math.log(T) - (10.0 + math.log(K0))
        Kc = math.exp(-(gB - gA))
        rho = P / (R_U * T) / sum((Y[k] if k > 1 else (yA if k == 0 else yB)) / W[k] for k in range(9))
        CA, CB = rho * yA / W[0], rho * yB / W[1]
        return W[1] * (kf * CA - kf / Kc * CB) / rho

    dt = 2e-4

    def rk4(nst):
        yB, hh = yB0, dt / nst
        for _ in range(nst):
            k1 = r(yB); k2 = r(yB + 0.5 * hh * k1); k3 = r(yB + 0.5 * hh * k2); k4 = r(yB + hh * k3)
            yB += hh / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        return yB

    ref_prev, nst = rk4(200), 400
    while True:
        ref = rk4(nst)
        if abs(ref - ref_prev) < 1e-14:
            break
        ref_prev, nst = ref, nst * 2
    T1, Y1, st, cnt, _ = om.integrate(np.array([T0]), np.array([P]), Y[:, None].copy(), dt,
                                      rtol=1e-10, atol=1e-14)
    assert st[0] == 0
    assert abs(Y1[1, 0] - ref) <= 1e-8 * abs(ref - yB0)
    assert abs(T1[0] - T_of(ref)) <= 1e-6
    assert abs(T1[0] - T0) > 10.0      # the case really moves T


def test_rk4_brute_force_mild_mechanism(tmp_path, oracle_lib):
    m = make_mechanism(seed=1, K=9, R=21, E=3, logA_range=(2.0, 6.0))
    om = _oracle_for(m, tmp_path, oracle_lib)
    f = cells4096(m, n=16, seed=33)
    dt = 1e-6
    T1, Y1, st, cnt, _ = om.integrate(f.T, f.p, f.Y, dt, rtol=1e-11, atol=1e-16)
    assert np.all(st == 0)
    for i in range(16):
        y0 = np.append(f.Y[:, i], f.T[i])
        prev, _ = om.rk4(P, y0, dt, 8)
        n = 16
        while True:
            cur, bad = om.rk4(P, y0, dt, n)
            assert bad == 0
            if np.max(np.abs(cur - prev) / (np.abs(cur) + 1e-14)) < 1e-12:
                break
            prev, n = cur, n * 2
        assert abs(T1[i] - cur[-1]) <= 1e-8 * cur[-1]
        assert np.all(np.abs(Y1[:, i] - cur[:-1]) <= 1e-9 * np.abs(cur[:-1]) + 1e-14)


# --------------------------------------------------------------------------- invariants

def test_conservation_and_tolerance_convergence(om9, mech_dir):
    from chemgen.mechanism import read_mechanism
    m = read_mechanism(str(mech_dir / "M9.mech"))
    f = cells4096(m, n=128, seed=77)
    W = m.molar_masses()
    res = {}
    for rtol in (1e-6, 1e-8, 1e-10, 1e-12):
        T1, Y1, st, cnt, _ = om9.integrate(f.T, f.p, f.Y, f.dt, rtol=rtol, atol=rtol * 1e-4)
        assert np.all(st == 0)
        res[rtol] = (T1, Y1)
        for i in range(0, 128, 7):
            b0 = m.counts.T @ (f.Y[:, i] / W)
            b1 = m.counts.T @ (Y1[:, i] / W)
            assert np.allclose(b1, b0, rtol=1e-12, atol=1e-14)
            h0 = om9.enthalpy(f.T[i], f.Y[:, i])
            h1 = om9.enthalpy(T1[i], Y1[:, i])
            cp = np.sum(Y1[:, i] * om9.thermo(T1[i])[0] * R_U / W)
            assert abs(h1 - h0) / cp <= 10 * rtol * T1[i]
    d = [np.abs(res[a][0] - res[1e-12][0]).max() for a in (1e-6, 1e-8, 1e-10)]
    assert d[0] > d[1] > d[2]
    assert d[2] < 1e-5


def test_standard_tolerances_vs_tight_reference(om9, mech_dir):
    """Error of the standard settings (rtol 1e-8, atol 1e-12) against a run at
    rtol 1e-13 stays at the tolerance level (reported beside parity results)."""
    from chemgen.mechanism import read_mechanism
    m = read_mechanism(str(mech_dir / "M9.mech"))
    f = cells4096(m, n=64)
    T1, Y1, st, _, _ = om9.integrate(f.T, f.p, f.Y, f.dt)
    T2, Y2, st2, _, _ = om9.integrate(f.T, f.p, f.Y, f.dt, rtol=1e-13, atol=1e-17, max_steps=100000)
    assert np.all(st == 0) and np.all(st2 == 0)
    assert np.abs(T1 - T2).max() <= 1e-8 * 2500 * 10
    assert np.abs(Y1 - Y2).max() <= 1e-6


def test_failure_restores_input(om9, mech_dir):
    from chemgen.mechanism import read_mechanism
    m = read_mechanism(str(mech_dir / "M9.mech"))
    f = cells4096(m, n=8)
    T1, Y1, st, cnt, _ = om9.integrate(f.T, f.p, f.Y, f.dt, max_steps=1)
    busy = cnt[:, 0] >= 1
    assert np.all(st[busy] == 1)
    assert np.array_equal(T1[busy], f.T[busy]) and np.array_equal(Y1[:, busy], f.Y[:, busy])
    Tn = f.T.copy()
    Tn[3] = float("nan")
    T2, Y2, st2, _, _ = om9.integrate(Tn, f.p, f.Y, f.dt)
    assert st2[3] == 4 and np.isnan(T2[3])
    assert np.all(st2[np.arange(8) != 3] == 0)


def test_equilibrium_cells_take_one_step(om9, mech_dir):
    from chemgen.mechanism import read_mechanism
    m = read_mechanism(str(mech_dir / "M9.mech"))
    g = flame_field(m, (8, 8, 8), 102, 1e-6, "t", "M9")
    ends = np.where((g.c < 1e-12) | (g.c > 1 - 1e-12))[0]
    T1, Y1, st, cnt, _ = om9.integrate(g.T[ends], g.p[ends], g.Y[:, ends], 1e-6)
    assert np.all(st == 0) and np.all(cnt[:, 0] <= 2)


def test_maximum_order_option(oracle_lib):
    """qmax caps the order the step selection may raise to: on y' = -y the
    accepted steps fall strictly with the cap (the step size grows with the
    order of the local error), every cap meets the tolerance-scaled error of
    the exact solution, and qmax = 5 is the default method bit for bit."""
    f = lambda t, y: -y
    j = lambda t, y: np.array([[-1.0]])
    exact = math.exp(-2.0)
    steps = []
    for q in (1, 2, 3, 4, 5):
        y, st, c = oracle_lib.bdf_user(f, j, [1.0], 2.0, rtol=1e-6, atol=1e-14, qmax=q)
        assert st == 0
        assert abs(y[0] - exact) <= 1e3 * 1e-6 * exact
        steps.append(int(c[0]))
    assert all(a > b for a, b in zip(steps, steps[1:])), steps
    y5, _, c5 = oracle_lib.bdf_user(f, j, [1.0], 2.0, rtol=1e-6, atol=1e-14)
    y5q, _, c5q = oracle_lib.bdf_user(f, j, [1.0], 2.0, rtol=1e-6, atol=1e-14, qmax=5)
    assert y5[0] == y5q[0] and np.array_equal(c5, c5q)


def test_maximum_order_option_on_cells(om9, mech_dir):
    """The same option through the cell integrator: a lower cap never takes
    fewer steps, and the results stay within the tolerance-scaled distance of
    the default method's."""
    from chemgen.fields import cells4096
    from chemgen.mechanism import read_mechanism
    f = cells4096(read_mechanism(str(mech_dir / "M9.mech")), n=64, seed=7)
    T5, Y5, s5, c5, _ = om9.integrate(f.T, f.p, f.Y, f.dt)
    T2, Y2, s2, c2, _ = om9.integrate(f.T, f.p, f.Y, f.dt, qmax=2)
    assert np.all(s5 == 0) and np.all(s2 == 0)
    assert np.all(c2[:, 0] >= c5[:, 0]) and c2[:, 0].sum() > c5[:, 0].sum()
    assert np.max(np.abs(T2 - T5)) < 1e-3


def test_initial_step_and_first_step_error_closed_form(oracle_lib):
    """Step selection pinned on y' = lam y, y(0) = 1 (a linear problem, so the
    difference quotient of the initial-step estimate is exact):
      * h0 = 0.5 sqrt(2 / (lam^2 w)), w = 1 / (rtol + atol): half the step
        whose second-derivative error estimate equals the tolerance;
      * the first step is backward Euler from the Taylor start (Nordsieck
        (1, h lam)): its correction is e = (h lam)^2 / (1 - h lam) and, with
        no past steps, the error constant is 1/2, so dsm_1 = |e| w / 2; this
        estimate equals the true local error exp(h lam) - 1/(1 - h lam) to
        leading order in h lam;
      * that error, dsm_1 = 1/4, asks for a step factor (6 dsm_1)^(-1/2) < 1.5,
        so the second step keeps h_1."""
    for lam, rtol, atol in ((-1.0, 1e-6, 1e-12), (-250.0, 1e-8, 1e-14), (3.0, 1e-7, 1e-12)):
        f = lambda t, y, lam=lam: lam * y
        j = lambda t, y, lam=lam: np.array([[lam]])
        y, st, c, tr = oracle_lib.bdf_user_trace(f, j, [1.0], 40.0 / abs(lam), rtol=rtol, atol=atol)
        assert st == 0 and tr.shape[0] == c[0]
        w = 1.0 / (rtol + atol)
        h0 = 0.5 * math.sqrt(2.0 / (lam * lam * w))
        assert tr[0, 1] == pytest.approx(h0, rel=1e-12)
        assert tr[0, 0] == pytest.approx(h0, rel=1e-15) and tr[0, 2] == 1
        x = h0 * lam
        e = x * x / (1.0 - x)
        assert tr[0, 3] == pytest.approx(0.5 * abs(e) * w, rel=1e-9)
        true_err = abs(math.exp(x) - 1.0 / (1.0 - x))
        assert (tr[0, 3] / w) / true_err == pytest.approx(1.0, abs=3 * abs(x))
        assert tr[0, 3] == pytest.approx(0.25, rel=1e-2)
        assert tr[1, 1] == tr[0, 1]


def test_order_sequence_on_smooth_decay(oracle_lib):
    """Order selection on y' = -y over [0, 25] at tight tolerances (a smooth
    solution, where higher orders pay): the order starts at 1, changes by one
    at a time, is kept at least q + 1 steps after each change (2 at the
    start), climbs to the cap, and every accepted step meets the tolerance;
    the cap itself is honoured.  Step sizes, between accepted steps whose
    successor passed at its first attempt: h never shrinks; a change is at
    least a factor 1.5 and at most 10 (1e4 after the first step); where the
    order stays and h changes below the cap, the same-order error predicted
    for the new step, dsm (h_new/h)^(q+1), is one sixth of the tolerance
    (safety factor 6).  The last step lands on t_end."""
    f = lambda t, y: -y
    j = lambda t, y: np.array([[-1.0]])
    for qmax in (5, 3):
        y, st, c, tr = oracle_lib.bdf_user_trace(f, j, [1.0], 25.0, rtol=1e-10, atol=1e-16, qmax=qmax)
        assert st == 0
        q = tr[:, 2].astype(int)
        assert q[0] == 1 and q.max() == qmax and q.min() >= 1
        assert np.all(np.abs(np.diff(q)) <= 1)
        change = np.where(np.diff(q) != 0)[0] + 1          # first step at a new order
        runs = np.diff(np.concatenate([[0], change]))        # lengths of the completed runs
        assert runs[0] >= 2
        assert np.all(runs[1:] >= q[change[:-1]] + 1), (q.tolist(),)
        assert np.all(tr[:, 3] <= 1.0)
        assert abs(y[0] - math.exp(-25.0)) <= 1e2 * 1e-10 * math.exp(-25.0) + 1e-14
        assert tr[-1, 0] == 25.0
        ratio = tr[1:-1, 1] / tr[:-2, 1]                    # last step clipped to t_end: excluded
        clean = tr[1:-1, 4] == 0
        assert clean.sum() >= 0.9 * ratio.size
        cap = np.where(np.arange(ratio.size) == 0, 1e4, 10.0)
        ok = (ratio == 1.0) | ((ratio >= 1.5 * (1 - 1e-12)) & (ratio <= cap * (1 + 1e-12)))
        assert np.all(ok[clean])
        same = clean & (q[1:-1] == q[:-2]) & (ratio != 1.0) & (ratio < cap * (1 - 1e-12))
        pred = 6.0 * tr[:-2, 3] * ratio ** (q[:-2] + 1)
        assert same.sum() >= 5
        assert np.allclose(pred[same], 1.0, rtol=1e-4), pred[same]


def _lambda_coeffs(xi, q):
    """Coefficients (ascending) of prod_{i=1..q} (1 + x / xi_i)."""
    c = np.array([1.0])
    for i in range(1, q + 1):
        c = np.convolve(c, [1.0, 1.0 / xi[i]])
    return c


@pytest.mark.parametrize("q", [2, 3, 4, 5])
def test_order_change_keeps_the_interpolated_values(oracle_lib, q):
    """The Nordsieck order change, checked as polynomials in x = (t - t_n)/h:
    lowering to q - 1 keeps the values at x = 0 and at the q - 1 most recent
    past points x = -xi_i and drops the degree-q term; raising to q + 1 keeps
    the values at x = 0 and at the q past points and adds exactly
    e (x / xi_{q+1}) prod_{i<=q} (1 + x / xi_i)."""
    rng = np.random.default_rng(q)
    N = 3
    xi = np.zeros(q + 2)
    xi[1] = 1.0
    for i in range(2, q + 2):
        xi[i] = xi[i - 1] + rng.uniform(0.3, 2.0)
    z = rng.normal(size=(q + 2, N))
    z[q + 1] = 0.0
    lam = _lambda_coeffs(xi, q)
    e = rng.normal(size=N)

    def P(zz, deg, x):
        return sum(zz[k] * x ** k for k in range(deg + 1))

    down = oracle_lib.order_change(q, q - 1, xi, lam, e, z[: q + 1])
    for x in [0.0] + [-xi[i] for i in range(1, q)]:
        assert np.allclose(P(down, q - 1, x), P(z, q, x), rtol=1e-12, atol=1e-12)
    up = oracle_lib.order_change(q, q + 1, xi, lam, e, z)
    for x in [0.0] + [-xi[i] for i in range(1, q + 1)]:
        assert np.allclose(P(up, q + 1, x), P(z, q, x), rtol=1e-12, atol=1e-12)
    added = np.convolve([0.0, 1.0 / xi[q + 1]], lam)     # (x / xi_{q+1}) Lambda_q(x)
    assert np.allclose(up[: q + 2] - z[: q + 2], np.outer(added, e), rtol=1e-13, atol=1e-14)
