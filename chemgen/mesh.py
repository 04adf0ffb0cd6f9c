"""Seeded structured box meshes in the owner/neighbour (ldu) face addressing.

Input building only: cell centres, face geometry and the face lists of a
hexahedral box, stored the way a finite-volume code with ldu matrices keeps
them (the paper's Section 3.1 and its ldu/CSR figure): internal faces in
upper-triangular order (owner < neighbour, sorted by owner, then by
neighbour), each with its linear-interpolation weight, the inverse distance
between the two cell centres and its area; and six boundary patches (x-, x+,
y-, y+, z-, z+), each a list of the cells next to its faces with the face
areas and the inverse centre-to-face distances.  Coordinates may be
stretched (geometric grading) so that interpolation weights differ from
one half.  No discretisation arithmetic happens here: the Laplacian's
coefficients are computed by the oracle and by the GPU library.
"""
from __future__ import annotations

import dataclasses
from typing import List

import numpy as np

#: Boundary condition types of a patch (as stored in the mesh's patch_type).
FIXED_VALUE, ZERO_GRADIENT = 0, 1


@dataclasses.dataclass
class BoxMesh:
    shape: tuple                  # (nx, ny, nz)
    centres: np.ndarray           # (ncells, 3)
    owner: np.ndarray             # (nfaces,) int32
    neighbour: np.ndarray         # (nfaces,) int32
    weight: np.ndarray            # (nfaces,) owner weight of linear interpolation
    delta: np.ndarray             # (nfaces,) 1 / |C_neighbour - C_owner|
    mag_sf: np.ndarray            # (nfaces,) face area
    patch_start: np.ndarray       # (npatches + 1,) int64 offsets into the boundary-face arrays
    face_cells: np.ndarray        # (nbfaces,) int32 cell next to each boundary face
    bdelta: np.ndarray            # (nbfaces,) 1 / |face centre - cell centre|
    bmag_sf: np.ndarray           # (nbfaces,) face area
    bcentres: np.ndarray          # (nbfaces, 3) boundary face centres
    patch_type: np.ndarray        # (npatches,) int32 FIXED_VALUE / ZERO_GRADIENT

    @property
    def ncells(self) -> int:
        return int(self.centres.shape[0])

    @property
    def nfaces(self) -> int:
        return int(self.owner.size)

    @property
    def nbfaces(self) -> int:
        return int(self.face_cells.size)


def _graded(n: int, length: float, ratio: float) -> np.ndarray:
    """n + 1 node coordinates on [0, length], consecutive spacings in geometric
    progression with last/first spacing = ratio."""
    if n == 1 or ratio == 1.0:
        return np.linspace(0.0, length, n + 1)
    g = ratio ** (1.0 / (n - 1))
    d = g ** np.arange(n)
    return np.concatenate([[0.0], np.cumsum(d)]) * (length / d.sum())


def box_mesh(nx: int, ny: int, nz: int, lengths=(1.0, 1.0, 1.0), grading=(1.0, 1.0, 1.0),
             patch_types=(FIXED_VALUE, FIXED_VALUE, ZERO_GRADIENT, ZERO_GRADIENT, FIXED_VALUE, ZERO_GRADIENT)
             ) -> BoxMesh:
    """Structured box of nx x ny x nz hexahedra, cell index i + nx (j + ny k)."""
    xs = [_graded(n, L, r) for n, L, r in zip((nx, ny, nz), lengths, grading)]
    cs = [0.5 * (x[1:] + x[:-1]) for x in xs]
    K, J, I = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    I, J, K = I.ravel(), J.ravel(), K.ravel()
    cell = (I + nx * (J + ny * K)).astype(np.int64)
    centres = np.stack([cs[0][I], cs[1][J], cs[2][K]], axis=1)
    dx = [np.diff(x) for x in xs]                 # cell widths per axis
    own, nei, w, dl, sf = [], [], [], [], []
    # candidate faces of every cell towards +x, +y, +z; sorted by (owner, neighbour)
    for axis, (step, last, idx) in enumerate(((1, nx - 1, I), (nx, ny - 1, J), (nx * ny, nz - 1, K))):
        m = idx < last
        o = cell[m]
        n_ = o + step
        c_o = centres[o, axis]
        c_n = centres[n_, axis]
        face = xs[axis][idx[m] + 1]               # face position along the axis
        own.append(o)
        nei.append(n_)
        w.append((c_n - face) / (c_n - c_o))
        dl.append(1.0 / (c_n - c_o))
        other = [a for a in range(3) if a != axis]
        sf.append(dx[other[0]][[I, J, K][other[0]][m]] * dx[other[1]][[I, J, K][other[1]][m]])
    own = np.concatenate(own)
    nei = np.concatenate(nei)
    order = np.lexsort((nei, own))
    fc, bd, bs, bcen = [], [], [], []
    starts = [0]
    for axis in range(3):
        idx = [I, J, K][axis]
        n_ax = (nx, ny, nz)[axis]
        other = [a for a in range(3) if a != axis]
        for side in (0, 1):
            m = idx == (0 if side == 0 else n_ax - 1)
            c = cell[m]
            face = xs[axis][0 if side == 0 else n_ax]
            fc.append(c)
            bd.append(1.0 / np.abs(face - centres[c, axis]))
            bs.append(dx[other[0]][[I, J, K][other[0]][m]] * dx[other[1]][[I, J, K][other[1]][m]])
            p = centres[c].copy()
            p[:, axis] = face
            bcen.append(p)
            starts.append(starts[-1] + c.size)
    return BoxMesh((nx, ny, nz), centres, own[order].astype(np.int32), nei[order].astype(np.int32),
                   np.concatenate(w)[order], np.concatenate(dl)[order], np.concatenate(sf)[order],
                   np.array(starts, dtype=np.int64), np.concatenate(fc).astype(np.int32), np.concatenate(bd),
                   np.concatenate(bs), np.concatenate(bcen), np.asarray(patch_types, dtype=np.int32))


def laplacian_fields(mesh: BoxMesh, seed: int):
    """Seeded smooth diffusivity gamma > 0 per cell and per boundary face,
    and boundary values psi_b (the inputs of the Laplacian assembly)."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.5, 1.5, size=3)
    ph = rng.uniform(0.0, 2 * np.pi, size=3)

    def g(p):
        return 1.0 + 0.5 * np.sin(2 * np.pi * a[0] * p[:, 0] + ph[0]) * np.cos(2 * np.pi * a[1] * p[:, 1] + ph[1]) \
            + 0.25 * np.sin(2 * np.pi * a[2] * p[:, 2] + ph[2])

    gamma_c = g(mesh.centres)
    gamma_b = g(mesh.bcentres)
    psi_b = rng.uniform(-1.0, 1.0, size=mesh.nbfaces)
    return gamma_c, gamma_b, psi_b
