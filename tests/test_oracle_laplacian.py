"""Pins of the Laplacian-assembly oracle (paper Section 3.1, Algorithm 1, and
the ldu/CSR figure) against facts other than its own formula: the
7-point stencil of a uniform grid with constant diffusivity, exactness of
the finite-volume flux balance on linear fields (stretched grids included),
symmetry and zero row sums away from fixed-value boundaries, the scipy
sparse matrix built from the same entries, and the CSR product equal to the
ldu product."""
import numpy as np
import pytest

from chemgen.mesh import FIXED_VALUE, ZERO_GRADIENT, box_mesh, laplacian_fields
from oracle import laplacian as L


def test_uniform_grid_is_the_seven_point_stencil():
    """gamma = 1 on a uniform grid of spacing h: every interior row is
    h (psi_E + psi_W + psi_N + psi_S + psi_T + psi_B - 6 psi_P), the
    finite-difference Laplacian times the cell volume."""
    n, h = 6, 1.0 / 6
    m = box_mesh(n, n, n)
    g = np.ones(m.ncells)
    lo, up, dg, ic, bc = L.assemble(m, g, np.ones(m.nbfaces), np.zeros(m.nbfaces))
    assert np.allclose(up, h) and np.array_equal(up, lo)
    idx = lambda i, j, k: i + n * (j + n * k)
    psi = np.random.default_rng(1).normal(size=m.ncells)
    out = L.operator_apply(m, lo, up, dg, ic, bc, psi)
    for (i, j, k) in [(1, 1, 1), (2, 3, 4), (4, 4, 1)]:
        c = idx(i, j, k)
        fd = sum(psi[idx(*t)] for t in [(i + 1, j, k), (i - 1, j, k), (i, j + 1, k), (i, j - 1, k),
                                        (i, j, k + 1), (i, j, k - 1)]) - 6 * psi[c]
        assert out[c] == pytest.approx(h * fd, rel=1e-12)


@pytest.mark.parametrize("grading", [(1.0, 1.0, 1.0), (3.0, 0.4, 1.7)])
def test_linear_fields_balance_exactly(grading):
    """Constant gamma, psi linear in x, y, z and the exact values on every
    boundary (all patches fixed-value): the fluxes through each cell's faces
    cancel, L(psi) = 0 in every cell, on uniform and graded grids."""
    m = box_mesh(7, 5, 4, lengths=(2.0, 1.0, 0.5), grading=grading, patch_types=(FIXED_VALUE,) * 6)
    a = np.array([0.7, -1.3, 2.1])
    psi = m.centres @ a + 0.4
    psi_b = m.bcentres @ a + 0.4
    g = 2.5
    lo, up, dg, ic, bc = L.assemble(m, np.full(m.ncells, g), np.full(m.nbfaces, g), psi_b)
    out = L.operator_apply(m, lo, up, dg, ic, bc, psi)
    scale = np.abs(up).max() * np.abs(psi).max()
    assert np.abs(out).max() <= 1e-12 * scale


def test_symmetry_row_sums_and_zero_gradient():
    """lower == upper; with only zero-gradient patches every row sums to
    zero (constants are in the null space) and the source vanishes."""
    m = box_mesh(5, 4, 3, grading=(2.0, 1.0, 0.5), patch_types=(ZERO_GRADIENT,) * 6)
    gc, gb, pb = laplacian_fields(m, 3)
    lo, up, dg, ic, bc = L.assemble(m, gc, gb, pb)
    assert np.array_equal(lo, up)
    out = L.operator_apply(m, lo, up, dg, ic, bc, np.full(m.ncells, 3.7))
    assert np.abs(out).max() <= 1e-13 * np.abs(dg).max()
    assert not ic.any() and not bc.any()


def test_csr_matches_scipy_and_ldu_product():
    """The CSR form against scipy.sparse built from (row, column, value)
    triples of the definition, and its product against the ldu product."""
    import scipy.sparse as sp
    m = box_mesh(6, 5, 4, grading=(1.5, 0.7, 2.0))
    gc, gb, pb = laplacian_fields(m, 4)
    lo, up, dg, ic, bc = L.assemble(m, gc, gb, pb)
    rp, col, val, rhs = L.to_csr(m, lo, up, dg, ic, bc)
    own, nei = m.owner.astype(np.int64), m.neighbour.astype(np.int64)
    d = dg.copy()
    np.add.at(d, m.face_cells.astype(np.int64), ic)
    A = sp.coo_matrix((np.concatenate([up, lo, d]), (np.concatenate([own, nei, np.arange(m.ncells)]),
                                                      np.concatenate([nei, own, np.arange(m.ncells)])))).tocsr()
    A.sort_indices()
    assert np.array_equal(A.indptr, rp) and np.array_equal(A.indices, col) and np.allclose(A.data, val, rtol=0)
    assert all(np.all(np.diff(col[rp[i]:rp[i + 1]]) > 0) for i in range(m.ncells))
    psi = np.random.default_rng(7).normal(size=m.ncells)
    a = L.operator_apply(m, lo, up, dg, ic, bc, psi)
    b = L.csr_apply(rp, col, val, rhs, psi)
    assert np.allclose(a, b, rtol=1e-13, atol=1e-13 * np.abs(a).max())
