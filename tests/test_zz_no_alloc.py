"""chem_integrate_noalloc: the integrator entry point that allocates no
device memory (its start-pass workspace is a fixed per-GPU array).  Called
through the C ABI and compared with chem_integrate on the same inputs: the
same kernels run, so outputs, per-cell status and counters are equal bit for
bit, on two calls in a row, the second smaller, and beyond the fixed array's
size the call fails cleanly."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


def _say(msg):
    print(msg, flush=True)


def _run(torch, mech, f, sel, entry, opts=None):
    dev = "cuda:0"
    T = torch.tensor(np.ascontiguousarray(f.T[sel]), dtype=torch.float64, device=dev)
    p = torch.tensor(np.ascontiguousarray(f.p[sel]), dtype=torch.float64, device=dev)
    Y = torch.tensor(np.ascontiguousarray(f.Y[:, sel]), dtype=torch.float64, device=dev)
    st = torch.full((sel.size,), -1, dtype=torch.int32, device=dev)
    cn = torch.zeros(6 * sel.size, dtype=torch.int32, device=dev)
    getattr(mech, entry)(T, p, Y, f.dt, opts=opts, status=st, counters=cn)
    torch.cuda.synchronize()
    return T.cpu().numpy(), Y.cpu().numpy(), st.cpu().numpy(), cn.cpu().numpy()


@pytest.mark.parametrize("schedule", [-1, 2])
def test_noalloc_equals_integrate(torch, mech_dir, schedule):
    from chemgen.fields import flame64, seeded_sample
    from chemgen.mechanism import read_mechanism
    from paper_2312_13513_amd import chem
    m = read_mechanism(str(mech_dir / "M9.mech"))
    f = flame64(m)
    mech = chem.Mechanism(str(mech_dir / "M9.mech"), 0)
    o = chem.chem_default_opts()
    o.schedule = schedule
    # two calls in a row, the second smaller: 20,000 then 3,001 cells of the
    # 64^3 flame field (the second reuses the fixed array the first filled)
    for n_cells, seed in ((20000, 21), (3001, 22)):
        sel = seeded_sample(f.n, n_cells, seed=seed)
        _say(f"[noalloc schedule {schedule}] {n_cells} cells")
        a = _run(torch, mech, f, sel, "integrate_noalloc", o)
        b = _run(torch, mech, f, sel, "integrate", o)
        for x, y, name in zip(a, b, ("T", "Y", "status", "counters")):
            assert np.array_equal(x, y), f"{name} differs from chem_integrate ({n_cells} cells)"
        assert np.all(a[2] == 0)
    mech.close()


def test_noalloc_rejects_beyond_fixed_array(torch, mech_dir):
    from paper_2312_13513_amd import chem
    mech = chem.Mechanism(str(mech_dir / "M9.mech"), 0)
    n = 340000   # above floor((2^25 - 1276) / (8 K + 28)) = 335,531 and the exact bound for K = 9
    dev = "cuda:0"
    T = torch.full((n,), 1200.0, dtype=torch.float64, device=dev)
    Y = torch.full((9, n), 1.0 / 9.0, dtype=torch.float64, device=dev)
    o = chem.chem_default_opts()
    o.schedule = 0
    with pytest.raises(chem.ChemError, match="fixed workspace"):
        mech.integrate_noalloc(T, T, Y, 1e-6, opts=o)
    # the refusal left the handle usable: a small call still matches
    from chemgen.fields import cells4096
    from chemgen.mechanism import read_mechanism
    f = cells4096(read_mechanism(str(mech_dir / "M9.mech")), n=512)
    sel = np.arange(512)
    a = _run(torch, mech, f, sel, "integrate_noalloc", o)
    b = _run(torch, mech, f, sel, "integrate", o)
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    mech.close()
