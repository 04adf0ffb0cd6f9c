"""GPU parity of the implicit Laplacian assembly (Section 3.1, Algorithm 1)
and of the ldu -> CSR conversion, and of the direct CSR assembly (no
atomics, deterministic), through the C ABI, against the numpy oracle on the
same seeded meshes and fields.

Bars: the CSR pattern is integer data and must be equal.  upper and lower
are five or six roundings (u = 2^-53) on each side, fused differently
(interpolation as an FMA on the GPU): within 12 u = 1.3e-15 relative, taken
as 1.5e-15; the diagonal adds up to six such terms with atomics, in an
order that changes from run to run: within 2.5e-15 of the sum of the
magnitudes of its terms; the boundary coefficients (two or three
roundings) within 1e-15 relative."""
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


def _run(torch, m, seed):
    from chemgen.mesh import laplacian_fields
    from paper_2312_13513_amd import chem
    gc, gb, pb = laplacian_fields(m, seed)
    dev = torch.device("cuda:0")
    t = lambda a: torch.tensor(a, dtype=torch.float64, device=dev)
    g = chem.LduMesh(m)
    z = lambda n: torch.full((max(n, 1),), float("nan"), dtype=torch.float64, device=dev)
    lo, up, dg, ic, bc = z(m.nfaces), z(m.nfaces), z(m.ncells), z(m.nbfaces), z(m.nbfaces)
    g.laplacian(t(gc), t(gb), t(pb), lo, up, dg, ic, bc)
    val, rhs = z(g.nnz), z(m.ncells)
    g.to_csr(lo, up, dg, ic, bc, val, rhs)
    rp = torch.zeros(m.ncells + 1, dtype=torch.int32, device=dev)
    col = torch.zeros(g.nnz, dtype=torch.int32, device=dev)
    g.csr_pattern(rp, col)
    # the direct CSR assembly, twice (no atomics: the same bits both times)
    val2, rhs2, val3, rhs3 = z(g.nnz), z(m.ncells), z(g.nnz), z(m.ncells)
    g.laplacian_csr(t(gc), t(gb), t(pb), val2, rhs2)
    g.laplacian_csr(t(gc), t(gb), t(pb), val3, rhs3)
    torch.cuda.synchronize()
    assert torch.equal(val2, val3) and torch.equal(rhs2, rhs3)
    out = {k: v.cpu().numpy() for k, v in (("lower", lo), ("upper", up), ("diag", dg), ("internal", ic),
                                            ("boundary", bc), ("val", val), ("rhs", rhs), ("row_ptr", rp),
                                            ("col", col), ("val_direct", val2), ("rhs_direct", rhs2))}
    out["lower"], out["upper"] = out["lower"][:m.nfaces], out["upper"][:m.nfaces]
    out["internal"], out["boundary"] = out["internal"][:m.nbfaces], out["boundary"][:m.nbfaces]
    g.close()
    return (gc, gb, pb), out


def _compare(tag, m, fields, out, dbar=2.5e-15):
    """dbar: the diagonal's bar relative to the sum of its terms' magnitudes
    (two summation orders of n terms differ by at most 2 (n - 1) u of it)."""
    from oracle import laplacian as L
    lo, up, dg, ic, bc = L.assemble(m, *fields)
    rp, col, val, rhs = L.to_csr(m, lo, up, dg, ic, bc)
    assert np.array_equal(out["row_ptr"], rp) and np.array_equal(out["col"], col)
    rel = lambda a, b: np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)) if a.size else 0.0
    e_up, e_lo = rel(out["upper"], up), rel(out["lower"], lo)
    gross = np.zeros(m.ncells)
    np.add.at(gross, m.owner.astype(np.int64), np.abs(up))
    np.add.at(gross, m.neighbour.astype(np.int64), np.abs(lo))
    e_dg = np.max(np.abs(out["diag"] - dg) / np.maximum(gross, 1e-300))
    e_b = max(rel(out["internal"], ic), rel(out["boundary"], bc))
    dcsr = np.abs(out["val"] - val)
    _say(f"[{tag}] cells {m.ncells} faces {m.nfaces} nnz {rp[-1]}: upper {e_up:.1e} lower {e_lo:.1e} "
         f"diag {e_dg:.1e} boundary {e_b:.1e} csr max|d| {dcsr.max():.1e}")
    assert e_up <= 1.5e-15 and e_lo <= 1.5e-15 and e_b <= 1e-15 and e_dg <= dbar
    assert np.array_equal(out["lower"], out["upper"])
    # the CSR values are the GPU's own ldu values moved (off-diagonals
    # bitwise), diagonal entries and rhs within the diagonal's bar
    rows = np.repeat(np.arange(m.ncells), np.diff(rp))
    diag_entry = col == rows
    # off-diagonal entries: the GPU's upper/lower values moved, so within the
    # upper/lower bar of the oracle; diagonal entries within the diagonal's
    assert np.max(np.abs(out["val"][~diag_entry] - val[~diag_entry]) /
                  np.maximum(np.abs(val[~diag_entry]), 1e-300), initial=0.0) <= 1.5e-15
    dscale = gross + np.abs(val[diag_entry])
    assert np.max(np.abs(out["val"][diag_entry] - val[diag_entry]) / np.maximum(dscale, 1e-300)) <= dbar
    # rhs: a sum of up to three boundary terms of either sign, measured
    # against the sum of their magnitudes
    rgross = np.zeros(m.ncells)
    np.add.at(rgross, m.face_cells.astype(np.int64), np.abs(bc))
    assert np.max(np.abs(out["rhs"] - rhs) / np.maximum(rgross, 1e-300)) <= 2.5e-15
    # direct CSR assembly: off-diagonals are the same face coefficients as
    # the ldu path (bitwise), diagonal and rhs within the same bars
    vd = out["val_direct"]
    assert np.array_equal(vd[~diag_entry], out["val"][~diag_entry])
    assert np.max(np.abs(vd[diag_entry] - val[diag_entry]) / np.maximum(dscale, 1e-300)) <= dbar
    assert np.max(np.abs(out["rhs_direct"] - rhs) / np.maximum(rgross, 1e-300)) <= 2.5e-15


@pytest.mark.parametrize("shape,grading", [((13, 9, 7), (2.0, 0.5, 1.3)), ((1, 1, 1), (1.0, 1.0, 1.0)),
                                           ((64, 1, 1), (3.0, 1.0, 1.0)), ((17, 16, 15), (1.0, 1.0, 1.0))])
def test_parity_small_meshes(torch, shape, grading):
    from chemgen.mesh import FIXED_VALUE, ZERO_GRADIENT, box_mesh
    m = box_mesh(*shape, grading=grading,
                 patch_types=(FIXED_VALUE, ZERO_GRADIENT, FIXED_VALUE, FIXED_VALUE, ZERO_GRADIENT, FIXED_VALUE))
    fields, out = _run(torch, m, 5)
    _compare(f"ldu-{shape}", m, fields, out)


def _hub_mesh():
    """A graded box plus extra faces that join ten hub cells to up to 60
    others each (owner < neighbour, upper-triangular order kept): rows of up
    to 68 entries, two of which reach past the edge of the 1024-entry block
    holding their diagonal (one 21 entries past its end, one 46 before its
    start), beyond the direct assembly's 16-entry LDS halo."""
    import dataclasses

    from chemgen.mesh import box_mesh
    m = box_mesh(16, 12, 6, grading=(1.5, 1.0, 0.8))
    rng = np.random.default_rng(11)
    pairs = set(zip(m.owner.tolist(), m.neighbour.tolist()))
    own, nei = m.owner.tolist(), m.neighbour.tolist()
    w, d, s = m.weight.tolist(), m.delta.tolist(), m.mag_sf.tolist()
    for hub in (184, 418, 427, 446, 592, 932, 934, 1007, 1076, 1097):
        for o in rng.choice(m.ncells, size=60, replace=False).tolist():
            a, b = min(hub, o), max(hub, o)
            if a == b or (a, b) in pairs:
                continue
            pairs.add((a, b))
            own.append(a)
            nei.append(b)
            w.append(rng.uniform(0.2, 0.8))
            d.append(rng.uniform(1.0, 20.0))
            s.append(rng.uniform(0.01, 0.1))
    order = np.lexsort((np.array(nei), np.array(own)))
    arr = lambda x, t: np.asarray(x, dtype=t)[order]
    return dataclasses.replace(m, owner=arr(own, np.int32), neighbour=arr(nei, np.int32), weight=arr(w, np.float64),
                               delta=arr(d, np.float64), mag_sf=arr(s, np.float64))


def test_parity_long_rows(torch):
    """Rows longer than a block's halo, crossing block edges both ways: the
    direct assembly's diagonal takes the far entries from the coefficient
    array.  Diagonal bar from the longest row's term count."""
    m = _hub_mesh()
    fields, out = _run(torch, m, 8)
    rp, col = out["row_ptr"].astype(np.int64), out["col"].astype(np.int64)
    before = after = 0
    for i in range(m.ncells):
        b, e = rp[i], rp[i + 1]
        dp = b + int(np.searchsorted(col[b:e], i))
        j0 = dp // 1024 * 1024
        before, after = max(before, j0 - b), max(after, e - (j0 + 1024))
    assert before > 16 and after > 16   # the cases the test is for
    nterms = int(np.diff(rp).max()) + 3
    _compare("ldu-hub", m, fields, out, dbar=2 * (nterms - 1) * 2.0 ** -53)


def test_csr_product_matches_operator(torch):
    """The GPU's CSR matrix and right-hand side reproduce the operator of the
    ldu arrays (oracle's product definition) on a random field."""
    from chemgen.mesh import box_mesh
    from oracle import laplacian as L
    m = box_mesh(11, 10, 9, grading=(1.7, 1.0, 0.6))
    fields, out = _run(torch, m, 6)
    psi = np.random.default_rng(2).normal(size=m.ncells)
    a = L.operator_apply(m, out["lower"], out["upper"], out["diag"], out["internal"], out["boundary"], psi)
    b = L.csr_apply(out["row_ptr"].astype(np.int64), out["col"].astype(np.int64), out["val"], out["rhs"], psi)
    assert np.allclose(a, b, rtol=1e-13, atol=1e-13 * np.abs(a).max())


def test_parity_128_cubed(torch):
    """The benchmark's mesh (128^3 cells, graded in x and z, fixed-value and
    zero-gradient patches): every coefficient against the oracle."""
    from chemgen.mesh import box_mesh
    m = box_mesh(128, 128, 128, grading=(2.0, 1.0, 0.5))
    fields, out = _run(torch, m, 7)
    _compare("ldu-128^3", m, fields, out)


def test_rejects_bad_meshes(torch):
    from chemgen.mesh import box_mesh
    from paper_2312_13513_amd import chem
    m = box_mesh(3, 3, 3)
    m.owner[[4, 5]] = m.owner[[5, 4]]
    m.neighbour[[4, 5]] = m.neighbour[[5, 4]]
    with pytest.raises(chem.ChemError, match="upper-triangular"):
        chem.LduMesh(m)
    m = box_mesh(3, 3, 3)
    m.neighbour[2] = m.owner[2]
    with pytest.raises(chem.ChemError, match="owner < neighbour"):
        chem.LduMesh(m)
    m = box_mesh(3, 3, 3)
    m.patch_type[1] = 7
    with pytest.raises(chem.ChemError, match="patch types"):
        chem.LduMesh(m)
