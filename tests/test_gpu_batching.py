"""Batching: integration of a listed subset in a given order, the LPT order,
and the autotuner.  The per-cell result does not depend on which lane or
wave takes the cell or when, so reordered and subset runs must be bitwise
equal to the plain run on the same cells."""
import numpy as np
import pytest

from test_gpu_integrate import DT_TOL, DY_TOL, _say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


def _dev(torch, a, dtype=None):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype or torch.float64, device="cuda:0")


@pytest.fixture(scope="module")
def m9(mech_dir, torch):
    from paper_2312_13513_amd import chem
    m = chem.Mechanism(str(mech_dir / "M9.mech"), 0)
    yield m
    m.close()


@pytest.fixture(scope="module")
def field(mech_dir):
    from chemgen.fields import cells4096
    from chemgen.mechanism import read_mechanism
    return cells4096(read_mechanism(str(mech_dir / "M9.mech")), n=3000, seed=12)


@pytest.mark.parametrize("schedule", [0, 1, 2])
def test_indexed_subset_is_bitwise_plain(torch, m9, field, schedule):
    from paper_2312_13513_amd import chem
    f = field
    o = chem.chem_default_opts()
    o.schedule = schedule
    rng = np.random.default_rng(5)
    sub = rng.choice(f.n, size=777, replace=False).astype(np.int32)   # random order
    # plain run of the subset as its own field
    Ts, Ys = _dev(torch, f.T[sub]), _dev(torch, f.Y[:, sub])
    cs = torch.zeros(6 * sub.size, dtype=torch.int32, device="cuda:0")
    m9.integrate(Ts, _dev(torch, f.p[sub]), Ys, f.dt, opts=o, counters=cs)
    # indexed run on the full arrays, with out-of-range entries mixed in
    idx = np.concatenate([sub[:400], [-1, f.n, 10 ** 9], sub[400:]]).astype(np.int32)
    T, Y = _dev(torch, f.T), _dev(torch, f.Y)
    st = torch.full((f.n,), -5, dtype=torch.int32, device="cuda:0")
    cnt = torch.full((6 * f.n,), -5, dtype=torch.int32, device="cuda:0")
    m9.integrate_indexed(T, _dev(torch, f.p), Y, _dev(torch, idx, torch.int32), f.dt, opts=o, status=st,
                         counters=cnt)
    torch.cuda.synchronize()
    T, Y, st, cnt = T.cpu().numpy(), Y.cpu().numpy(), st.cpu().numpy(), cnt.cpu().numpy().reshape(6, f.n)
    assert np.array_equal(T[sub], Ts.cpu().numpy()) and np.array_equal(Y[:, sub], Ys.cpu().numpy())
    assert np.array_equal(cnt[:, sub], cs.cpu().numpy().reshape(6, sub.size))
    rest = np.setdiff1d(np.arange(f.n), sub)
    assert np.array_equal(T[rest], f.T[rest]) and np.array_equal(Y[:, rest], f.Y[:, rest])
    assert np.all(st[rest] == -5) and np.all(st[sub] == 0)


def test_lpt_order_matches_stable_sort(torch):
    from paper_2312_13513_amd import chem
    rng = np.random.default_rng(6)
    for n in (1, 63, 1000, 70001):
        cost = rng.integers(0, 50, size=n).astype(np.int32)
        order = torch.zeros(n, dtype=torch.int32, device="cuda:0")
        chem.chem_lpt_order(_dev(torch, cost, torch.int32), order)
        ref = np.argsort(-cost.astype(np.int64), kind="stable")
        assert np.array_equal(order.cpu().numpy(), ref)


def test_lpt_ordered_run_is_bitwise_plain(torch, m9, field):
    f = field
    T1, Y1 = _dev(torch, f.T), _dev(torch, f.Y)
    p = _dev(torch, f.p)
    cnt = torch.zeros(6 * f.n, dtype=torch.int32, device="cuda:0")
    m9.integrate(T1, p, Y1, f.dt, counters=cnt)
    from paper_2312_13513_amd import chem
    order = torch.zeros(f.n, dtype=torch.int32, device="cuda:0")
    chem.chem_lpt_order(cnt[:f.n].contiguous(), order)
    T2, Y2 = _dev(torch, f.T), _dev(torch, f.Y)
    m9.integrate_indexed(T2, p, Y2, order, f.dt)
    torch.cuda.synchronize()
    assert torch.equal(T1, T2) and torch.equal(Y1, Y2)


def test_autotune_choice_meets_parity(torch, m9, field, om9):
    from paper_2312_13513_amd import chem
    f = field
    T, Y, p = _dev(torch, f.T), _dev(torch, f.Y), _dev(torch, f.p)
    best, lpt, ms = m9.autotune(T, p, Y, f.dt, max_sample=2048)
    _say(f"[autotune] schedule {best.schedule} jac_batch {best.jac_batch} lpt {lpt} {ms:.3f} ms on 2048 cells")
    assert best.schedule in (0, 1, 2) and ms > 0
    # the states passed in are not modified
    assert np.array_equal(T.cpu().numpy(), f.T) and np.array_equal(Y.cpu().numpy(), f.Y)
    o = chem.chem_default_opts()
    o.schedule = -2
    m9.integrate(T, p, Y, f.dt, opts=o)
    torch.cuda.synchronize()
    To, Yo, _, _, _ = om9.integrate(f.T, f.p, f.Y, f.dt)
    dT = np.abs(T.cpu().numpy() - To).max()
    dY = np.abs(Y.cpu().numpy() - Yo).max()
    _say(f"[autotune] tuned run vs oracle: max|dT| {dT:.3e} K max|dY| {dY:.3e}")
    assert dT < DT_TOL and dY < DY_TOL


def _time_opts(torch, mech, T0, p, Y0, dt, o, reps=3):
    """Best of reps HIP-event timings of one call (state restored each time)."""
    import torch as t
    best = 1e30
    for _ in range(reps):
        T, Y = T0.clone(), Y0.clone()
        a, b = t.cuda.Event(enable_timing=True), t.cuda.Event(enable_timing=True)
        a.record()
        mech.integrate(T, p, Y, dt, opts=o)
        b.record()
        t.cuda.synchronize()
        best = min(best, a.elapsed_time(b))
    return best


def test_autotune_picks_the_fastest_at_full_size(torch, m9, mech_dir):
    """On a 131,072-cell flame field (the default sample is then the whole
    field) the tuned choice is, within 10 %, the fastest of every candidate
    configuration timed again at full size; the measured table lists every
    candidate once."""
    from chemgen.fields import flame_field
    from chemgen.mechanism import read_mechanism
    from paper_2312_13513_amd import chem
    m = read_mechanism(str(mech_dir / "M9.mech"))
    f = flame_field(m, (64, 64, 32), seed=44, dt=1e-6, name="flame64x32", mech_name="M9")
    T, Y, p = _dev(torch, f.T), _dev(torch, f.Y), _dev(torch, f.p)
    best, lpt, ms = m9.autotune(T, p, Y, f.dt)
    table = m9.autotune_results()
    _say(f"[autotune-full] chose schedule {best.schedule} jac_batch {best.jac_batch} waves/SIMD "
         f"{best.waves_per_simd} lpt {lpt}: {ms:.3f} ms; table {[(e['schedule'], e['jac_batch'], e['lpt'], e['waves_per_simd'], round(e['ms'], 3)) for e in table]}")
    keys = [(e["schedule"], e["jac_batch"], e["lpt"], e["waves_per_simd"]) for e in table]
    assert len(keys) == len(set(keys)) and len(keys) == 3 + 8
    assert min(e["ms"] for e in table) == pytest.approx(ms)
    times = {}
    order = torch.empty(f.n, dtype=torch.int32, device="cuda:0")
    for sched, jb, l, w in keys:
        if l:
            continue    # LPT runs need the order of a previous step; natural order suffices here
        o = chem.chem_default_opts()
        o.schedule, o.jac_batch, o.waves_per_simd = sched, jb, w
        times[(sched, jb, w)] = _time_opts(torch, m9, T, p, Y, f.dt, o)
    _say(f"[autotune-full] full-size times {times}")
    chosen = times.get((best.schedule, best.jac_batch, best.waves_per_simd))
    if chosen is not None:
        assert chosen <= 1.10 * min(times.values())


def test_tuned_choice_per_size_class_and_cache_file(torch, mech_dir, field, tmp_path, monkeypatch):
    """Choices are kept per size class; with CHEM_TUNE_CACHE set they are
    written to that file and a new handle of the same mechanism file restores
    them: schedule -2 then runs the tuned schedule (bitwise equal to asking
    for it explicitly)."""
    from paper_2312_13513_amd import chem
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("CHEM_TUNE_CACHE", str(cache))
    f = field
    a = chem.Mechanism(str(mech_dir / "M9.mech"), 0)
    n1, n2 = 1000, 3000
    T, Y, p = _dev(torch, f.T[:n2]), _dev(torch, f.Y[:, :n2]), _dev(torch, f.p[:n2])
    b1 = a.autotune(T[:n1].contiguous(), p[:n1].contiguous(), Y[:, :n1].contiguous(), f.dt)[0]
    b2 = a.autotune(T, p, Y, f.dt)[0]
    a.close()
    lines = cache.read_text().splitlines()
    assert len(lines) == 2 and all(ln.startswith("chemtune1 gfx") for ln in lines)
    assert [int(ln.split()[5]) for ln in lines] == [9, 11]
    b = chem.Mechanism(str(mech_dir / "M9.mech"), 0)
    for n, bst in ((n1, b1), (n2, b2)):
        o = chem.chem_default_opts()
        o.schedule = -2
        T1, Y1 = _dev(torch, f.T[:n]), _dev(torch, f.Y[:, :n])
        b.integrate(T1, p[:n].contiguous(), Y1, f.dt, opts=o)
        o2 = chem.chem_default_opts()
        o2.schedule = bst.schedule
        T2, Y2 = _dev(torch, f.T[:n]), _dev(torch, f.Y[:, :n])
        b.integrate(T2, p[:n].contiguous(), Y2, f.dt, opts=o2)
        torch.cuda.synchronize()
        assert torch.equal(T1, T2) and torch.equal(Y1, Y2)
    b.close()


def test_stats_totals_match_the_per_cell_outputs(torch, m9, field):
    """chem_get_stats against numpy sums of the same per-cell arrays, with
    failed cells (a NaN state, a step cap) among them."""
    from paper_2312_13513_amd import chem
    f = field
    n = 1500
    T = f.T[:n].copy()
    T[3] = float("nan")
    o = chem.chem_default_opts()
    o.max_steps = 3
    Tg, Yg, p = _dev(torch, T), _dev(torch, f.Y[:, :n]), _dev(torch, f.p[:n])
    st = torch.full((n,), -1, dtype=torch.int32, device="cuda:0")
    cn = torch.zeros(6 * n, dtype=torch.int32, device="cuda:0")
    m9.integrate(Tg, p, Yg, f.dt, opts=o, status=st, counters=cn)
    fb = torch.tensor([17], dtype=torch.int64, device="cuda:0")
    s = chem.chem_get_stats(st, cn, n, fallback_count=fb)
    sn, c = st.cpu().numpy(), cn.cpu().numpy().reshape(6, n)
    _say(f"[stats] {s}")
    assert s["cells"] == n and s["fallback_cells"] == 17
    assert s["steps_total"] == c[0].sum() and s["rhs_evals"] == c[1].sum()
    assert s["jac_evals"] == c[2].sum() and s["newton_iters"] == c[3].sum()
    assert s["rejects"] == c[4].sum() + c[5].sum() and s["steps_max"] == c[0].max()
    assert s["status_count"] == [int(np.sum(sn == k)) for k in range(8)]
    assert s["status_count"][4] >= 1 and s["status_count"][1] >= 1
    # status only, counters only, and no cells
    s2 = chem.chem_get_stats(st, None, n)
    assert s2["status_count"] == s["status_count"] and s2["steps_total"] == 0
    s3 = chem.chem_get_stats(None, cn, n)
    assert s3["steps_total"] == s["steps_total"] and sum(s3["status_count"]) == 0
    s4 = chem.chem_get_stats(st, cn, 0)
    assert s4["cells"] == 0 and s4["steps_total"] == 0 and sum(s4["status_count"]) == 0
