"""GPU parity of the tile schedule (16 lanes per cell, four cells per wave,
mechanisms with N = K + 1 <= 16): against the CPU oracle on the 9-species
mechanism, and against the wave schedule, which takes the same decisions with
the same operations per cell (the compiler may fuse multiply-adds differently
in the two kernels, so agreement is at round-off, not bitwise).  Ragged cell
counts (not a multiple of four) and index lists with entries outside the
arrays must reproduce the full tile run bit for bit; failure statuses and the
FP32 Jacobian/LU mode are covered."""
import numpy as np
import pytest

from test_gpu_integrate import compare, compare_cell_envelope, compare_flips_to_oracle_alternatives, run_gpu, _say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


@pytest.fixture(scope="module")
def g9(mech_dir, torch):
    from paper_2312_13513_amd import chem
    m = chem.Mechanism(str(mech_dir / "M9.mech"), 0)
    yield m
    m.close()


@pytest.fixture(scope="module")
def field(mech_dir):
    from chemgen.fields import cells4096
    from chemgen.mechanism import read_mechanism
    return cells4096(read_mechanism(str(mech_dir / "M9.mech")), n=3001, seed=21)


def _opts(schedule, precision=0, max_steps=None):
    from paper_2312_13513_amd import chem
    o = chem.chem_default_opts()
    o.schedule = schedule
    o.precision = precision
    if max_steps is not None:
        o.max_steps = max_steps
    return o


@pytest.fixture(scope="module")
def tile_and_wave(torch, g9, field):
    f = field
    tile = run_gpu(torch, g9, f.T, f.p, f.Y, f.dt, opts=_opts(2))
    wave = run_gpu(torch, g9, f.T, f.p, f.Y, f.dt, opts=_opts(1))
    return tile, wave


def _bitwise(a, b):
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_tile_matches_oracle(tile_and_wave, field, om9):
    f = field
    Tg, Yg, sg, cg = tile_and_wave[0]
    To, Yo, so, co, _ = om9.integrate(f.T, f.p, f.Y, f.dt)
    flips = compare_flips_to_oracle_alternatives("tile-M9", om9, f.T, f.p, f.Y, f.dt, Tg, Yg, sg, cg, To, Yo, so, co)
    assert flips.size <= 3


def test_tile_agrees_with_wave(tile_and_wave):
    tile, wave = tile_and_wave
    compare("tile-vs-wave", *tile, *wave)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 67])
def test_tile_ragged_sizes(torch, g9, field, tile_and_wave, n):
    f = field
    out = run_gpu(torch, g9, f.T[:n], f.p[:n], f.Y[:, :n], f.dt, opts=_opts(2))
    full = tile_and_wave[0]
    _bitwise(out, (full[0][:n], full[1][:, :n], full[2][:n], full[3][:n]))


def test_tile_index_list(torch, g9, field, tile_and_wave):
    f = field
    dev = "cuda:0"
    rng = np.random.default_rng(3)
    sub = rng.choice(f.n, size=501, replace=False).astype(np.int32)
    idx = np.concatenate([sub[:200], [-1, f.n, 1 << 30], sub[200:]]).astype(np.int32)
    T = torch.tensor(f.T, dtype=torch.float64, device=dev)
    Y = torch.tensor(f.Y, dtype=torch.float64, device=dev)
    st = torch.full((f.n,), -5, dtype=torch.int32, device=dev)
    g9.integrate_indexed(T, torch.tensor(f.p, dtype=torch.float64, device=dev), Y,
                         torch.tensor(idx, dtype=torch.int32, device=dev), f.dt, opts=_opts(2), status=st)
    torch.cuda.synchronize()
    T, Y, st = T.cpu().numpy(), Y.cpu().numpy(), st.cpu().numpy()
    full = tile_and_wave[0]
    assert np.array_equal(T[sub], full[0][sub]) and np.array_equal(Y[:, sub], full[1][:, sub])
    rest = np.setdiff1d(np.arange(f.n), sub)
    assert np.array_equal(T[rest], f.T[rest]) and np.all(st[rest] == -5) and np.all(st[sub] == 0)


def test_tile_failure_statuses(torch, g9, field, tile_and_wave):
    f = field
    sel = np.arange(0, 130)
    T = f.T[sel].copy()
    T[7] = float("nan")
    for opts in (_opts(2, max_steps=1), _opts(2)):
        tile = run_gpu(torch, g9, T, f.p[sel], f.Y[:, sel], f.dt, opts=opts)
        opts.schedule = 1
        wave = run_gpu(torch, g9, T, f.p[sel], f.Y[:, sel], f.dt, opts=opts)
        assert np.array_equal(tile[2], wave[2])
        assert tile[2][7] == 4 and np.isnan(tile[0][7])
    many = tile_and_wave[0][3][sel, 0] > 1
    capped = run_gpu(torch, g9, T, f.p[sel], f.Y[:, sel], f.dt, opts=_opts(2, max_steps=1))
    assert np.all(capped[2][many & (sel != 7)] == 1)


def test_tile_fp32_lu_error(torch, g9, field, om9):
    """FP32 Jacobian and LU, FP64 residual and state: the same error scale as
    the wave schedule's mixed mode against the FP64 oracle."""
    f = field
    n = 1024
    tile = run_gpu(torch, g9, f.T[:n], f.p[:n], f.Y[:, :n], f.dt, opts=_opts(2, precision=1))
    wave = run_gpu(torch, g9, f.T[:n], f.p[:n], f.Y[:, :n], f.dt, opts=_opts(1, precision=1))
    To, Yo = om9.integrate(f.T[:n], f.p[:n], f.Y[:, :n], f.dt)[:2]
    assert np.all(tile[2] == 0) and np.all(wave[2] == 0)
    dT, dY = np.abs(tile[0] - To).max(), np.abs(tile[1] - Yo).max()
    dTw = np.abs(wave[0] - To).max()
    _say(f"[tile] FP32 J/LU: max|dT| vs FP64 oracle {dT:.3e} K (wave schedule {dTw:.3e} K), max|dY| {dY:.3e}")
    assert dT < 1e-3 and dY < 1e-6


def test_tile_rejects_large_mechanism(torch, mech_dir):
    from paper_2312_13513_amd import chem
    g = chem.Mechanism(str(mech_dir / "M35.mech"), 0)
    T = torch.full((4,), 1500.0, dtype=torch.float64, device="cuda:0")
    Y = torch.full((35, 4), 1.0 / 35, dtype=torch.float64, device="cuda:0")
    with pytest.raises(chem.ChemError, match="tile"):
        g.integrate(T, T, Y, 1e-6, opts=_opts(2))
    g.close()


@pytest.fixture(scope="module")
def m15_path(tmp_path_factory):
    """A 15-species / 80-reaction synthetic mechanism: N = 16 fills a tile, and
    its tables plus the reaction scratch of four cells exceed what the tile
    kernel stages in LDS, so the kernel reads them from global memory."""
    from chemgen.mechanism import make_mechanism
    p = tmp_path_factory.mktemp("m15") / "M15.mech"
    make_mechanism(seed=11, K=15, R=80, E=3).write(str(p))
    return p


def test_tile_full_width_unstaged_tables(torch, m15_path, oracle_lib):
    from chemgen.fields import cells4096
    from chemgen.mechanism import read_mechanism
    from paper_2312_13513_amd import chem
    mpy = read_mechanism(str(m15_path))
    f = cells4096(mpy, n=515, seed=31)
    g = chem.Mechanism(str(m15_path), 0)
    om = oracle_lib.OracleMech(str(m15_path))
    tile = run_gpu(torch, g, f.T, f.p, f.Y, f.dt, opts=_opts(2))
    wave = run_gpu(torch, g, f.T, f.p, f.Y, f.dt, opts=_opts(1))
    To, Yo, so, co, _ = om.integrate(f.T, f.p, f.Y, f.dt)
    # random states of a random mechanism, up to 345 steps per cell: the
    # oracle's own ulp spread is the bar, cell by cell
    compare_cell_envelope("tile-M15", om, f.T, f.p, f.Y, f.dt, *tile, To, Yo, so, co)
    assert np.array_equal(tile[2], wave[2])
    g.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_refresh_deferral_is_bitwise_plain(torch, g9, mech_dir, precision):
    """From 65,536 queued cells the tile kernel lets a cell that needs a new
    Newton matrix wait a pass for a second cell of its wave (scheduling only).
    The whole 64^3 flame field (262,144 cells, deferral on) gives bit for bit
    the state, status and counters of the same cells run as five index lists
    of under 65,536 cells each (the plain loop)."""
    from chemgen.fields import flame64
    from chemgen.mechanism import read_mechanism
    f = flame64(read_mechanism(str(mech_dir / "M9.mech")))
    n = f.n
    assert n >= 4 * 65536
    full = run_gpu(torch, g9, f.T, f.p, f.Y, f.dt, opts=_opts(2, precision))
    dev = torch.device("cuda:0")
    T = torch.tensor(f.T, dtype=torch.float64, device=dev)
    p = torch.tensor(f.p, dtype=torch.float64, device=dev)
    Y = torch.tensor(np.ascontiguousarray(f.Y), dtype=torch.float64, device=dev)
    st = torch.full((n,), -1, dtype=torch.int32, device=dev)
    cn = torch.zeros(6 * n, dtype=torch.int32, device=dev)
    perm = np.random.default_rng(5).permutation(n).astype(np.int32)
    for part in np.array_split(perm, 5):
        assert part.size < 65536
        idx = torch.tensor(part, device=dev)
        g9.integrate_indexed(T, p, Y, idx, f.dt, opts=_opts(2, precision), status=st, counters=cn)
    torch.cuda.synchronize()
    parts = (T.cpu().numpy(), Y.cpu().numpy(), st.cpu().numpy(), cn.cpu().numpy().reshape(6, n).T)
    _say(f"[deferral precision={precision}] {n} cells: full run vs five index lists, steps mean {parts[3][:, 0].mean():.2f}")
    for a, b in zip(full, parts):
        assert a.shape == b.shape and np.array_equal(a, b)


def test_two_streams_global_scratch_bitwise_serial(torch, m15_path):
    """The 15-species / 80-reaction mechanism keeps its reaction scratch in
    global memory (tile and wave kernels).  Two calls in flight on two
    streams of the same handle take different scratch partitions: each gives
    bit for bit what it gives alone."""
    from chemgen.fields import cells4096
    from chemgen.mechanism import read_mechanism
    from paper_2312_13513_amd import chem
    mpy = read_mechanism(str(m15_path))
    fa = cells4096(mpy, n=1536, seed=41)
    fb = cells4096(mpy, n=1280, seed=42)
    g = chem.Mechanism(str(m15_path), 0)
    dev = torch.device("cuda:0")

    def state(f):
        return (torch.tensor(f.T, dtype=torch.float64, device=dev), torch.tensor(f.p, dtype=torch.float64, device=dev),
                torch.tensor(np.ascontiguousarray(f.Y), dtype=torch.float64, device=dev),
                torch.full((f.n,), -1, dtype=torch.int32, device=dev), torch.zeros(6 * f.n, dtype=torch.int32, device=dev))

    for schedule in (2, 1):
        alone = []
        for f in (fa, fb):
            T, p, Y, st, cn = state(f)
            g.integrate(T, p, Y, f.dt, opts=_opts(schedule), status=st, counters=cn)
            torch.cuda.synchronize()
            alone.append([x.cpu().numpy() for x in (T, Y, st, cn)])
        sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
        A, B = state(fa), state(fb)
        torch.cuda.synchronize()
        for s, (T, p, Y, st, cn), f in ((sa, A, fa), (sb, B, fb)):
            with torch.cuda.stream(s):
                g.integrate(T, p, Y, f.dt, opts=_opts(schedule), status=st, counters=cn, stream=s)
        torch.cuda.synchronize()
        for got, ref in zip((A, B), alone):
            T, p, Y, st, cn = got
            for x, r in zip((T, Y, st, cn), ref):
                assert np.array_equal(x.cpu().numpy(), r)
        _say(f"[two streams, schedule {schedule}] 1536 + 1280 cells in flight together equal the serial runs")
    g.close()
