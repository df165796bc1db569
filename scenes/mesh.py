"""Seeded synthetic tetrahedral meshes (Kuhn grids) and their surface topology.

This module builds inputs only: node positions, tet connectivity and boundary
faces/edges.  It contains none of the solver's arithmetic (no distances, no
elasticity), so both the oracle and the GPU path can consume its output.
"""
from __future__ import annotations

import itertools

import numpy as np

# The six Kuhn simplices of the unit cube: each walks from corner (0,0,0) to
# corner (1,1,1) adding one axis at a time, in the order of a permutation.
_PERMS = list(itertools.permutations(range(3)))


def kuhn_cube(n: int, a: float, origin=(0.0, 0.0, 0.0)):
    """An n*n*n-cell cube of edge a*n, each cell split into 6 Kuhn tets."""
    return kuhn_box(n, n, n, a, origin)


def kuhn_box(nx: int, ny: int, nz: int, a: float, origin=(0.0, 0.0, 0.0)):
    """An nx*ny*nz-cell box of spacing a, each cell split into 6 Kuhn tets.

    Node index = i + (nx+1)*(j + (ny+1)*k) (x fastest).  Every tet is returned
    with positive orientation.  Returns (nodes [N,3] float64, tets [T,4] int32).
    """
    mx, my, mz = nx + 1, ny + 1, nz + 1
    idx = np.arange(mx * my * mz).reshape(mz, my, mx)  # idx[k, j, i]
    nodes = np.stack(
        [
            np.broadcast_to(np.arange(mx)[None, None, :], (mz, my, mx)),
            np.broadcast_to(np.arange(my)[None, :, None], (mz, my, mx)),
            np.broadcast_to(np.arange(mz)[:, None, None], (mz, my, mx)),
        ],
        axis=-1,
    ).reshape(-1, 3).astype(np.float64) * a
    nodes += np.asarray(origin, dtype=np.float64)

    # cells in (k, j, i) order so tets follow node order
    ck, cj, ci = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ci, cj, ck = ci.ravel(), cj.ravel(), ck.ravel()
    tets = []
    for perm in _PERMS:
        corner = np.zeros((3,), dtype=np.int64)
        verts = [idx[ck, cj, ci]]
        for ax in perm:
            corner[ax] += 1
            verts.append(idx[ck + corner[2], cj + corner[1], ci + corner[0]])
        tets.append(np.stack(verts, axis=1))
    # cell-major, 6 tets per cell
    tets = np.stack(tets, axis=1).reshape(-1, 4)
    tets = orient_positive(nodes, tets)
    return nodes, tets.astype(np.int32)


def orient_positive(nodes: np.ndarray, tets: np.ndarray) -> np.ndarray:
    """Swap the last two vertices of every tet whose signed volume is negative."""
    p = nodes[tets]
    e1, e2, e3 = p[:, 1] - p[:, 0], p[:, 2] - p[:, 0], p[:, 3] - p[:, 0]
    s = np.einsum("ij,ij->i", np.cross(e1, e2), e3)
    out = tets.copy()
    neg = s < 0
    out[neg, 2], out[neg, 3] = tets[neg, 3], tets[neg, 2]
    return out


def boundary_faces(tets: np.ndarray) -> np.ndarray:
    """Faces that belong to exactly one tet, as [F,3] vertex triples (sorted ids)."""
    t = tets.astype(np.int64)
    faces = np.concatenate([t[:, [1, 2, 3]], t[:, [0, 2, 3]], t[:, [0, 1, 3]], t[:, [0, 1, 2]]])
    faces.sort(axis=1)
    nmax = int(t.max()) + 1
    key = (faces[:, 0] * nmax + faces[:, 1]) * nmax + faces[:, 2]
    uk, inv, cnt = np.unique(key, return_inverse=True, return_counts=True)
    once = cnt[inv] == 1
    return faces[once].astype(np.int32)


def face_edges(faces: np.ndarray) -> np.ndarray:
    """Unique edges of a set of triangles, [E,2] with e0 < e1."""
    f = faces.astype(np.int64)
    e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [0, 2]]])
    e.sort(axis=1)
    e = np.unique(e, axis=0)
    return e.astype(np.int32)


def surface_vertices(faces: np.ndarray) -> np.ndarray:
    return np.unique(faces.ravel()).astype(np.int32)


# The 24 proper rotations of a cube, as integer 3x3 matrices.
def cube_rotations() -> list:
    mats = []
    for perm in _PERMS:
        for signs in itertools.product((1, -1), repeat=3):
            m = np.zeros((3, 3), dtype=np.int64)
            for r, c in enumerate(perm):
                m[r, c] = signs[r]
            if round(np.linalg.det(m)) == 1:
                mats.append(m)
    assert len(mats) == 24
    return mats
