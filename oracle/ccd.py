"""Plain FP64 CPU oracle for the collision side of the time step:
UpdateActiveSet (Algorithm 3) and MaxStepSize (Algorithm 1).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Algorithm 3 (Section 4.3): collect the surface primitive pairs that collide
along the straight path from the intersection-free state x to the target
x_hat, drop those already in the active set, give every vertex the earliest
collision time T_v among the new pairs it belongs to, keep a new pair only if
its own time is the earliest of at least one of its vertices (it enters with
lambda = 0, gamma = 1), and remove every constraint whose decay factor fell
below 0.01.  MaxStepSize (Algorithm 1) is the largest step along the same
path that stays intersection-free and, Neo-Hookean being non-invertible,
inversion-free.

The paper delegates the collision queries to a linear BVH broad phase and
ACCD narrow phase (Section 5).  Readings (listed in the design doc):
  * Primitives are the boundary triangles of the tet mesh, their edges and
    their vertices; a point-triangle pair shares no vertex, an edge-edge pair
    no endpoint.
  * Broad phase: a pair is a candidate when the swept boxes of its two
    primitives (over both endpoint states) come within delta of each other
    on every axis.  Here it is brute force over all pairs.
  * Narrow phase: additive CCD (Li, Kaufman and Jiang, "Codimensional
    Incremental Potential Contact", 2021) with separation ratio s = 0.1 and
    zero thickness: advance by steps that cannot close the gap given the
    relative displacement bound, and stop at the first step whose distance is
    below s times the initial one.  A pair "collides" when that time is below
    1; its collision time is that (conservative) time.
  * ACCD gives up after 10^4 steps (a pair sliding at a tiny distance): the
    pair then counts as colliding at the time reached, which is conservative.
    A pair at distance 0 at t = 0 collides at t = 0.
  * The inversion bound: per tet, the first t in (0, 1] with
    det(D_s(t)) = s det(D_s(0)) (s = 0.1 again), found by bisection between
    the roots of the cubic's derivative.
  * MaxStepSize is the smallest collision time over all candidate pairs and
    the smallest inversion bound over all tets, 1 if there is none.
  * "The earliest collision time" of a vertex is taken up to the times' own
    rounding: a pair is kept when T_i <= T_v (1 + 1e-9).  Pairs of a rigidly
    moving structured mesh are tied in exact arithmetic, and two FP64 ACCD
    codes place such ties 1e-16..1e-10 apart in either order.
  * An edge pair that is (near-)parallel at x (|e_a x e_b|^2 < 1e-8 |e_a|^2
    |e_b|^2, the test under which the linearization rejects a constraint) does
    not enter the active set, before the earliest-time filter; it still limits
    the step size.
"""
from __future__ import annotations

import numpy as np

from . import core

S_SEP = 0.1          # ACCD separation ratio
STEP_FRAC = 0.9      # ACCD step safety factor after the first step
MAX_ACCD_ITERS = 10_000   # steps per pair; a pair still running counts as colliding at the time reached
GAMMA_REMOVE = 0.01  # Algorithm 3: constraints with gamma below this are removed
TIE_REL = 1e-9       # a time within this relative distance of T_v counts as T_v


# ------------------------------------------------------------------ surface --

def surface(tets):
    """Boundary triangles (faces of exactly one tet, vertices ascending, rows
    sorted), their edges (ascending pairs, sorted) and vertices (sorted)."""
    t = np.asarray(tets, dtype=np.int64)
    faces = np.concatenate([t[:, [0, 1, 2]], t[:, [0, 1, 3]], t[:, [0, 2, 3]], t[:, [1, 2, 3]]])
    faces = np.sort(faces, axis=1)
    uniq, cnt = np.unique(faces, axis=0, return_counts=True)
    tris = uniq[cnt == 1]
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [0, 2]]])
    edges = np.unique(e, axis=0)
    verts = np.unique(tris)
    return tris, edges, verts


# --------------------------------------------------------------- broad phase --

def swept_boxes(x0, x1, prims):
    """Per primitive (rows of vertex ids) the box of its vertices at both states."""
    P = np.concatenate([x0[prims], x1[prims]], axis=1)     # [n, 2k, 3]
    return P.min(axis=1), P.max(axis=1)


def boxes_near(lo_a, hi_a, lo_b, hi_b, delta):
    """Boxes within delta of each other on every axis (all pairs a x b)."""
    ok = np.ones((len(lo_a), len(lo_b)), dtype=bool)
    for k in range(3):
        ok &= (lo_a[:, None, k] - delta <= hi_b[None, :, k]) & (lo_b[None, :, k] - delta <= hi_a[:, None, k])
    return ok


def _near_pairs(lo_a, hi_a, lo_b, hi_b, delta, upper=False, rows=1024):
    """All (a, b) index pairs whose boxes are near (a < b only when upper),
    in row-major order; all pairs are tested, a block of rows at a time."""
    ia, ib = [], []
    for r0 in range(0, len(lo_a), rows):
        ok = boxes_near(lo_a[r0:r0 + rows], hi_a[r0:r0 + rows], lo_b, hi_b, delta)
        a, b = np.nonzero(ok)
        a = a + r0
        if upper:
            keep = b > a
            a, b = a[keep], b[keep]
        ia.append(a)
        ib.append(b)
    return np.concatenate(ia), np.concatenate(ib)


def candidates(x0, x1, tris, edges, verts, delta):
    """Brute-force broad phase: PT rows (v, t0, t1, t2) and EE rows
    (a0, a1, b0, b1), each in canonical order (edge a before edge b)."""
    vlo, vhi = swept_boxes(x0, x1, verts[:, None])
    tlo, thi = swept_boxes(x0, x1, tris)
    vi, ti = _near_pairs(vlo, vhi, tlo, thi, delta)
    pt = np.column_stack([verts[vi], tris[ti]])
    share = (pt[:, 0] == pt[:, 1]) | (pt[:, 0] == pt[:, 2]) | (pt[:, 0] == pt[:, 3])
    pt = pt[~share]
    elo, ehi = swept_boxes(x0, x1, edges)
    ia, ib = _near_pairs(elo, ehi, elo, ehi, delta, upper=True)
    ee = np.column_stack([edges[ia], edges[ib]])
    share = ((ee[:, 0] == ee[:, 2]) | (ee[:, 0] == ee[:, 3]) | (ee[:, 1] == ee[:, 2]) | (ee[:, 1] == ee[:, 3]))
    ee = ee[~share]
    return pt.astype(np.int64), ee.astype(np.int64)


# -------------------------------------------------------------- narrow phase --

def _dist(kind, X):
    """Distance of each pair; X [n, 4, 3]."""
    if kind == "pt":
        d, _, _ = core.pt_closest(X[:, 0], X[:, 1], X[:, 2], X[:, 3])
    else:
        d, _, _ = core.ee_closest(X[:, 0], X[:, 1], X[:, 2], X[:, 3])
    return d


def accd(kind, X0, X1, s=S_SEP, t_max=1.0):
    """Additive CCD of each pair along X(t) = X0 + t (X1 - X0), t in [0, t_max].

    Returns (hit [n] bool, toc [n]): toc is the conservative collision time
    where hit, t_max elsewhere.  The common translation is removed from the
    displacements; l_p bounds how fast the distance can shrink (the largest
    displacement of a vertex of the first primitive plus that of the second:
    PT splits 1 | 3 vertices, EE 2 | 2).  With d0 the initial distance the
    target gap is s d0; the first step is (1 - s) d0 / l_p, later ones
    0.9 d / l_p.  The search stops when a step lands below the gap (the time
    before that step is returned) or passes t_max (no collision)."""
    n = len(X0)
    P = X1 - X0
    P = P - P.mean(axis=1, keepdims=True)
    norms = np.linalg.norm(P, axis=2)
    split = 1 if kind == "pt" else 2
    lp = norms[:, :split].max(axis=1) + norms[:, split:].max(axis=1)
    hit = np.zeros(n, dtype=bool)
    toc = np.full(n, t_max)
    X = X0.copy()
    d = _dist(kind, X)
    gap = s * d
    t = np.zeros(n)
    touching = d == 0.0
    hit[touching] = True
    toc[touching] = 0.0
    act = (lp > 0.0) & ~touching
    tl = np.where(act, (1.0 - s) * d / np.where(act, lp, 1.0), 0.0)
    first = np.ones(n, dtype=bool)
    for _ in range(MAX_ACCD_ITERS):
        idx = np.nonzero(act)[0]
        if len(idx) == 0:
            break
        X[idx] = X[idx] + tl[idx, None, None] * P[idx]
        d_new = _dist(kind, X[idx])
        stop = (~first[idx]) & (d_new < gap[idx])
        hit[idx[stop]] = True
        toc[idx[stop]] = t[idx[stop]]
        go = idx[~stop]
        t[go] = t[go] + tl[go]
        over = t[go] > t_max
        act[idx[stop]] = False
        act[go[over]] = False
        cont = go[~over]
        tl[cont] = STEP_FRAC * d_new[~stop][~over] / lp[cont]
        first[idx] = False
    else:
        # iteration cap: report a collision at the time reached (conservative)
        idx = np.nonzero(act)[0]
        hit[idx] = True
        toc[idx] = t[idx]
    return hit, toc


# ---------------------------------------------------------- active set update --

def canonical(kind, ids):
    """Canonical key of a PT row (p, sorted triangle) or an EE row (sorted
    edges, edge a before edge b)."""
    ids = np.asarray(ids, dtype=np.int64).reshape(-1, 4)
    if kind == "pt":
        return np.column_stack([ids[:, 0], np.sort(ids[:, 1:], axis=1)])
    a = np.sort(ids[:, :2], axis=1)
    b = np.sort(ids[:, 2:], axis=1)
    swap = (a[:, 0] > b[:, 0]) | ((a[:, 0] == b[:, 0]) & (a[:, 1] > b[:, 1]))
    first = np.where(swap[:, None], b, a)
    second = np.where(swap[:, None], a, b)
    return np.column_stack([first, second])


def colliding_pairs(x, xh, tris, edges, verts, delta, s=S_SEP):
    """Candidates and their ACCD times along x -> x_hat: ((pt, T_pt), (ee, T_ee))
    restricted to the colliding pairs (time below 1)."""
    pt, ee = candidates(x, xh, tris, edges, verts, delta)
    out = []
    for kind, ids in (("pt", pt), ("ee", ee)):
        if len(ids) == 0:
            out.append((ids.reshape(0, 4), np.zeros(0)))
            continue
        hit, toc = accd(kind, x[ids], xh[ids], s)
        out.append((ids[hit], toc[hit]))
    return out


def ee_parallel(x, ee, tol=1e-8):
    """|e_a x e_b|^2 < tol |e_a|^2 |e_b|^2 at x: the edge pairs whose distance
    gradient is not unique (the linearization rejects them)."""
    ee = np.asarray(ee, dtype=np.int64).reshape(-1, 4)
    ea = x[ee[:, 1]] - x[ee[:, 0]]
    eb = x[ee[:, 3]] - x[ee[:, 2]]
    cr = np.cross(ea, eb)
    return np.einsum("ij,ij->i", cr, cr) < tol * np.einsum("ij,ij->i", ea, ea) * np.einsum("ij,ij->i", eb, eb)


def earliest_filter(n_nodes, pt, T_pt, ee, T_ee):
    """Algorithm 3's filter: T_v = min over the new pairs containing v; a pair
    stays when its time equals T_v for at least one of its vertices, equality
    taken up to the times' own rounding (T_i <= T_v (1 + 1e-9))."""
    Tv = np.full(n_nodes, np.inf)
    for ids, T in ((pt, T_pt), (ee, T_ee)):
        for a in range(4):
            np.minimum.at(Tv, ids[:, a], T)
    keep = []
    for ids, T in ((pt, T_pt), (ee, T_ee)):
        k = np.zeros(len(ids), dtype=bool)
        for a in range(4):
            k |= T <= Tv[ids[:, a]] * (1.0 + TIE_REL)
        keep.append(k)
    return keep


def update_active_set(n_nodes, x, xh, tris, edges, verts, pt_c, ee_c, lam, gam, delta, s=S_SEP):
    """Algorithm 3.  pt_c, ee_c: the current constraints (PT first in lam and
    gam).  Returns (pt', ee', lam', gam', info): surviving current constraints
    in their order, then the new ones (PT, then EE, each in canonical order)."""
    (pt, T_pt), (ee, T_ee) = colliding_pairs(x, xh, tris, edges, verts, delta, s)
    n_coll = (len(pt), len(ee))
    # an edge pair (near-)parallel at x has no unique distance gradient and
    # cannot be linearized: it does not enter the set (it still limits the step)
    ok = ~ee_parallel(x, ee)
    ee, T_ee = ee[ok], T_ee[ok]
    # drop pairs already in the active set
    have_pt = {tuple(r) for r in canonical("pt", pt_c)}
    have_ee = {tuple(r) for r in canonical("ee", ee_c)}
    new_pt = np.array([tuple(r) not in have_pt for r in canonical("pt", pt)], dtype=bool)
    new_ee = np.array([tuple(r) not in have_ee for r in canonical("ee", ee)], dtype=bool)
    pt, T_pt, ee, T_ee = pt[new_pt], T_pt[new_pt], ee[new_ee], T_ee[new_ee]
    kpt, kee = earliest_filter(n_nodes, pt, T_pt, ee, T_ee)
    add_pt, add_ee = pt[kpt], ee[kee]
    n_pt = len(pt_c)
    lam = np.asarray(lam, dtype=np.float64)
    gam = np.asarray(gam, dtype=np.float64)
    keep_pt = gam[:n_pt] >= GAMMA_REMOVE
    keep_ee = gam[n_pt:] >= GAMMA_REMOVE
    pt_out = np.concatenate([np.asarray(pt_c, dtype=np.int64).reshape(-1, 4)[keep_pt], add_pt])
    ee_out = np.concatenate([np.asarray(ee_c, dtype=np.int64).reshape(-1, 4)[keep_ee], add_ee])
    lam_out = np.concatenate([lam[:n_pt][keep_pt], np.zeros(len(add_pt)), lam[n_pt:][keep_ee], np.zeros(len(add_ee))])
    gam_out = np.concatenate([gam[:n_pt][keep_pt], np.ones(len(add_pt)), gam[n_pt:][keep_ee], np.ones(len(add_ee))])
    info = dict(colliding_pt=n_coll[0], colliding_ee=n_coll[1], parallel_ee=int((~ok).sum()),
                new_pt=int(len(pt)), new_ee=int(len(ee)), added_pt=int(len(add_pt)), added_ee=int(len(add_ee)),
                removed=int((~keep_pt).sum() + (~keep_ee).sum()))
    return pt_out, ee_out, lam_out, gam_out, info


# ------------------------------------------------------------ max step size --

def _det3(A):
    return np.linalg.det(A)


def inversion_bound(rest_tets_x0, x1_tets, s=S_SEP):
    """Per tet the first t in (0, 1] where det D_s(t) / det D_s(0) falls to s, or 1.
    rest_tets_x0, x1_tets: [T, 4, 3] vertex positions at t = 0 and t = 1.
    The tets need not be positively oriented: the ratio is the same for either
    vertex order.  det D_s(t) is a cubic in t; between consecutive roots of its
    derivative it is monotone, so the first sign change of
    f(t) = sign(det D_s(0)) det D_s(t) - s |det D_s(0)| is bracketed and
    bisected (60 halvings, the lower end returned)."""
    D0 = (rest_tets_x0[:, 1:] - rest_tets_x0[:, :1]).transpose(0, 2, 1)
    D1 = (x1_tets[:, 1:] - x1_tets[:, :1]).transpose(0, 2, 1)
    dD = D1 - D0
    j0 = _det3(D0)
    # cubic coefficients by exact interpolation at four points
    ts = np.array([0.0, 1.0 / 3.0, 2.0 / 3.0, 1.0])
    vals = np.stack([_det3(D0 + t * dD) for t in ts], axis=1)
    V = np.vander(ts, 4)                          # rows t^3, t^2, t, 1
    coef = np.linalg.solve(V, vals.T).T           # [T, 4]
    out = np.ones(len(D0))

    sg = np.where(j0 < 0.0, -1.0, 1.0)

    def f(i, t):
        c = coef[i]
        return sg[i] * (((c[0] * t + c[1]) * t + c[2]) * t + c[3]) - s * abs(j0[i])

    for i in range(len(D0)):
        a, b, c = 3 * coef[i, 0], 2 * coef[i, 1], coef[i, 2]
        crit = []
        if a != 0.0:
            disc = b * b - 4 * a * c
            if disc >= 0.0:
                r = np.sqrt(disc)
                crit = sorted([(-b - r) / (2 * a), (-b + r) / (2 * a)])
        elif b != 0.0:
            crit = [-c / b]
        knots = [0.0] + [t for t in crit if 0.0 < t < 1.0] + [1.0]
        for lo, hi in zip(knots, knots[1:]):
            if f(i, hi) <= 0.0:
                for _ in range(60):
                    mid = 0.5 * (lo + hi)
                    if f(i, mid) > 0.0:
                        lo = mid
                    else:
                        hi = mid
                out[i] = lo
                break
    return out


def max_step_size(x, xh, tets, tris, edges, verts, delta, s=S_SEP):
    """MaxStepSize: min(1, collision times of all candidate pairs, inversion bounds)."""
    alpha = 1.0
    pt, ee = candidates(x, xh, tris, edges, verts, delta)
    for kind, ids in (("pt", pt), ("ee", ee)):
        if len(ids):
            hit, toc = accd(kind, x[ids], xh[ids], s)
            if hit.any():
                alpha = min(alpha, float(toc[hit].min()))
    t = np.asarray(tets, dtype=np.int64)
    alpha = min(alpha, float(inversion_bound(x[t], xh[t], s).min()))
    return alpha
