"""Plain numpy oracle of the implicit Laplacian assembly and of the ldu -> CSR
conversion.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline may call it; the GPU library never does.

What it follows (paper Section 3.1):
  * Algorithm 1, implicit discretisation of div(gamma grad psi) on a
    finite-volume mesh in owner/neighbour (ldu) addressing: per internal face
    the face diffusivity by linear interpolation, gamma_f = w gamma_owner +
    (1 - w) gamma_neighbour, the off-diagonal coefficients
    upper = lower = gamma_f delta_f |S_f| (delta_f the inverse distance
    between the two cell centres), and the diagonal accumulated from every
    face: diag[owner] -= upper, diag[neighbour] -= lower; then per boundary
    patch, by its type, the coefficients the boundary adds to the diagonal
    (internal) and to the source (boundary).  Reading of the boundary
    coefficients (the paper names them, not their values): a fixed-value
    face adds the flux gamma_b |S_b| delta_b (psi_b - psi_P), so internal =
    -gamma_b |S_b| delta_b and boundary = gamma_b |S_b| delta_b psi_b; a
    zero-gradient face adds nothing.  The assembled operator is then
    L(psi) = A psi + r with A = ldu(lower, diag + internal, upper) and r the
    summed boundary coefficients.
  * The ldu/CSR figure: the same matrix by rows, each row's columns in
    increasing order (lower entries, the diagonal, upper entries), with the
    boundary's internal coefficients added to the diagonal and the boundary
    coefficients gathered into the right-hand side vector r.
"""
from __future__ import annotations

import numpy as np


def assemble(mesh, gamma_c, gamma_b, psi_b):
    """Algorithm 1: (lower, upper, diag, internal, boundary)."""
    own, nei = mesh.owner.astype(np.int64), mesh.neighbour.astype(np.int64)
    gamma_f = mesh.weight * gamma_c[own] + (1.0 - mesh.weight) * gamma_c[nei]
    upper = gamma_f * mesh.delta * mesh.mag_sf
    lower = upper.copy()
    diag = np.zeros(mesh.ncells)
    np.add.at(diag, own, -upper)
    np.add.at(diag, nei, -lower)
    internal = np.zeros(mesh.nbfaces)
    boundary = np.zeros(mesh.nbfaces)
    for p, kind in enumerate(mesh.patch_type):
        s = slice(int(mesh.patch_start[p]), int(mesh.patch_start[p + 1]))
        if kind == 0:   # fixed value
            c = gamma_b[s] * mesh.bmag_sf[s] * mesh.bdelta[s]
            internal[s] = -c
            boundary[s] = c * psi_b[s]
    return lower, upper, diag, internal, boundary


def operator_apply(mesh, lower, upper, diag, internal, boundary, psi):
    """L(psi) = A psi + r from the ldu arrays (row by row definition)."""
    own, nei = mesh.owner.astype(np.int64), mesh.neighbour.astype(np.int64)
    out = diag * psi
    np.add.at(out, own, upper * psi[nei])
    np.add.at(out, nei, lower * psi[own])
    fc = mesh.face_cells.astype(np.int64)
    np.add.at(out, fc, internal * psi[fc] + boundary)
    return out


def to_csr(mesh, lower, upper, diag, internal, boundary):
    """(row_ptr, col, val, rhs): the matrix by rows, columns increasing."""
    n = mesh.ncells
    own, nei = mesh.owner.astype(np.int64), mesh.neighbour.astype(np.int64)
    d = diag.copy()
    fc = mesh.face_cells.astype(np.int64)
    np.add.at(d, fc, internal)
    rhs = np.zeros(n)
    np.add.at(rhs, fc, boundary)
    rows = np.concatenate([own, nei, np.arange(n)])
    cols = np.concatenate([nei, own, np.arange(n)])
    vals = np.concatenate([upper, lower, d])
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    return np.cumsum(row_ptr), cols, vals, rhs


def csr_apply(row_ptr, col, val, rhs, psi):
    out = rhs.copy()
    for i in range(row_ptr.size - 1):
        a, b = row_ptr[i], row_ptr[i + 1]
        out[i] += np.dot(val[a:b], psi[col[a:b]])
    return out
