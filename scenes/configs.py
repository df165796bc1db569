"""Seeded synthetic workloads shaped like the paper's contact scenes.

Each builder returns a plain dict of numpy arrays that describes one Newton
step of the augmented-Lagrangian subproblem: the mesh and its rest shape, the
intersection-free linearization point x, the current iterate x_hat, the
inertia target x_tilde, the step h, and the active constraint set (point-
triangle and edge-edge pairs, each with a multiplier lambda and a decay factor
gamma) with the penalty kappa and the offset delta.

Constraint pairs are chosen across bodies by a *proxy* proximity (vertex to
triangle centroid, edge midpoint to edge midpoint), closest first, ties broken
by (type, ids).  That proxy is a generator choice only; the solver's own
distance functions are not used here.
"""
from __future__ import annotations

import hashlib

import numpy as np
from scipy.spatial import cKDTree

from .mesh import boundary_faces, cube_rotations, face_edges, kuhn_box, kuhn_cube, surface_vertices

SEED_BASE = 20251215


def _rng(seed: int, stream: str) -> np.random.Generator:
    """Independent sub-stream per purpose (noise, lambda, material, ...)."""
    tag = int.from_bytes(hashlib.sha256(stream.encode()).digest()[:4], "little")
    return np.random.default_rng([SEED_BASE + seed, tag])


def _face_on_plane(faces, pos, axis, value, tol=1e-9):
    on = np.all(np.abs(pos[faces][:, :, axis] - value) < tol, axis=1)
    return faces[on]


class _Surface:
    """Triangles, edges and vertices of one flat contact surface of one body."""

    def __init__(self, faces):
        self.faces = faces.astype(np.int32)
        self.edges = face_edges(self.faces)
        self.verts = surface_vertices(self.faces)


def _pt_candidates(x, pts_side, tri_side, k):
    """(proxy distance, p, t0, t1, t2) for the k nearest triangle centroids of each point."""
    tri = tri_side.faces
    cen = x[tri].mean(axis=1)
    k = min(k, len(tri))
    tree = cKDTree(cen)
    dist, j = tree.query(x[pts_side.verts], k=k)
    dist = dist.reshape(len(pts_side.verts), k)
    j = j.reshape(len(pts_side.verts), k)
    p = np.repeat(pts_side.verts, k)
    t = tri[j.ravel()]
    return dist.ravel(), np.column_stack([p, t]).astype(np.int64)


def _ee_candidates(x, side_a, side_b, k):
    ea, eb = side_a.edges, side_b.edges
    mid_a = x[ea].mean(axis=1)
    mid_b = x[eb].mean(axis=1)
    k = min(k, len(eb))
    tree = cKDTree(mid_b)
    dist, j = tree.query(mid_a, k=k)
    dist = dist.reshape(len(ea), k)
    j = j.reshape(len(ea), k)
    ia = np.repeat(np.arange(len(ea)), k)
    jb = j.ravel()
    ids = np.column_stack([ea[ia], eb[jb]]).astype(np.int64)
    # drop nearly parallel edge pairs (sin^2 of the angle below 1e-4)
    da = x[ids[:, 1]] - x[ids[:, 0]]
    db = x[ids[:, 3]] - x[ids[:, 2]]
    cr = np.cross(da, db)
    s2 = np.einsum("ij,ij->i", cr, cr) / (np.einsum("ij,ij->i", da, da) * np.einsum("ij,ij->i", db, db))
    keep = s2 >= 1e-4
    return dist.ravel()[keep], ids[keep]


def _select(dist, ids, n, type_id):
    """n smallest proxies; ties broken by (type, ids) lexicographically."""
    if n > len(dist):
        raise ValueError(f"only {len(dist)} candidates for {n} constraints")
    keys = [ids[:, c] for c in range(ids.shape[1] - 1, -1, -1)]
    order = np.lexsort(keys + [np.full(len(dist), type_id), dist])
    return ids[order[:n]]


def _pick(x, interfaces, n_pt, n_ee):
    """Pick constraints over a list of (surface_a, surface_b) facing pairs."""
    n_pts_total = sum(len(a.verts) + len(b.verts) for a, b in interfaces)
    n_edges_total = sum(len(a.edges) for a, b in interfaces)
    kp = int(np.ceil(1.5 * n_pt / max(n_pts_total, 1))) + 6
    ke = int(np.ceil(2.5 * n_ee / max(n_edges_total, 1))) + 8
    while True:
        d_list, id_list = [], []
        for a, b in interfaces:
            for ps, ts in ((a, b), (b, a)):
                d, ids = _pt_candidates(x, ps, ts, kp)
                d_list.append(d)
                id_list.append(ids)
        dpt, ipt = np.concatenate(d_list), np.concatenate(id_list)
        d_list, id_list = [], []
        for a, b in interfaces:
            d, ids = _ee_candidates(x, a, b, ke)
            d_list.append(d)
            id_list.append(ids)
        dee, iee = np.concatenate(d_list), np.concatenate(id_list)
        if len(dpt) >= n_pt and len(dee) >= n_ee:
            break
        kp, ke = kp * 2, ke * 2  # widen the query until the count is met
    pt = _select(dpt, ipt, n_pt, 0)
    ee = _select(dee, iee, n_ee, 1)
    return pt.astype(np.int32), ee.astype(np.int32)


def _finish(name, seed, rest, tets, E, nu, rho, fixed, x, x_hat, x_tilde, dt, pt, ee, lam,
            kappa, delta, tol, extra=None):
    n_c = len(pt) + len(ee)
    sc = dict(
        name=name, seed=seed,
        rest=np.ascontiguousarray(rest, dtype=np.float64),
        tets=np.ascontiguousarray(tets, dtype=np.int32),
        E=np.ascontiguousarray(E, dtype=np.float64),
        nu=np.ascontiguousarray(nu, dtype=np.float64),
        rho=np.ascontiguousarray(rho, dtype=np.float64),
        fixed=np.ascontiguousarray(fixed, dtype=np.uint8),
        x=np.ascontiguousarray(x, dtype=np.float64),
        x_hat=np.ascontiguousarray(x_hat, dtype=np.float64),
        x_tilde=np.ascontiguousarray(x_tilde, dtype=np.float64),
        dt=float(dt),
        pt=np.ascontiguousarray(pt, dtype=np.int32).reshape(-1, 4),
        ee=np.ascontiguousarray(ee, dtype=np.int32).reshape(-1, 4),
        lam=np.ascontiguousarray(lam, dtype=np.float64),
        gamma=np.ones(n_c, dtype=np.float64),
        kappa=float(kappa), delta=float(delta), tol=float(tol),
    )
    if extra:
        sc.update(extra)
    return sc


def digest(scene: dict) -> str:
    """sha256 over every array and scalar of a scene, in key order."""
    h = hashlib.sha256()
    for k in sorted(scene):
        v = scene[k]
        h.update(k.encode())
        if isinstance(v, np.ndarray):
            h.update(str(v.dtype).encode())
            h.update(str(v.shape).encode())
            h.update(np.ascontiguousarray(v).tobytes())
        else:
            h.update(repr(v).encode())
    return h.hexdigest()


def _stack_two_cubes(n, gap, lateral=(0.0, 0.0)):
    """Two unit cubes of n^3 cells, the upper one offset by `gap` above the lower
    and shifted sideways by `lateral` (in cell widths)."""
    a = 1.0 / n
    lo, tl = kuhn_cube(n, a, (0.0, 0.0, 0.0))
    hi, th = kuhn_cube(n, a, (lateral[0] * a, lateral[1] * a, 1.0 + gap))
    nodes = np.concatenate([lo, hi])
    tets = np.concatenate([tl, th + len(lo)])
    faces = boundary_faces(tl)
    top = _Surface(_face_on_plane(faces, lo, 2, 1.0))
    bot = _Surface(_face_on_plane(faces, lo, 2, 0.0) + len(lo))
    n_surf = 2 * len(surface_vertices(faces))
    return a, nodes, tets, len(lo), top, bot, n_surf


def tiny(seed: int = 1, lateral=(0.0, 0.0), n: int = 4, n_pt: int = 25, n_ee: int = 40, material=None):
    """Two stacked unit cubes (4^3 cells each), upper cube 1e-3 above the lower.

    `lateral` shifts the upper cube sideways (in cells) so that point-triangle
    pairs also fall in the triangle interior; the default is the plain stack.
    `material`: None (Neo-Hookean), "snh" / "cor" (stable Neo-Hookean /
    corotated linear everywhere), "mixed" / "mixed_cor" (the upper cube stable
    Neo-Hookean / corotated linear) or "all3" (tets cycling through codes 0, 1, 2)."""
    a, rest, tets, n_lo, top, bot, _ = _stack_two_cubes(n, 1e-3, lateral)
    N, T = len(rest), len(tets)
    fixed = np.zeros(N, dtype=np.uint8)
    fixed[:n_lo][rest[:n_lo, 2] == 0.0] = 1
    x = rest.copy()
    noise = _rng(seed, "noise").normal(0.0, 0.01 * a, size=(N, 3))
    x_hat = x + noise * (1 - fixed)[:, None]
    pt, ee = _pick(x, [(top, bot)], n_pt, n_ee)
    lam = _rng(seed, "lambda").uniform(0.0, 100.0, size=len(pt) + len(ee))
    extra = None
    if material is not None:
        codes = {"snh": (1, 1), "cor": (2, 2), "mixed": (0, 1), "mixed_cor": (0, 2)}
        if material == "all3":
            mat = (np.arange(T) % 3).astype(np.int32)
        else:
            lo, up = codes[material]
            mat = np.full(T, lo, dtype=np.int32)
            mat[len(tets) // 2:] = up
        extra = {"material": mat}
    return _finish("tiny", seed, rest, tets, np.full(T, 1e5), np.full(T, 0.4), np.full(T, 1000.0),
                   fixed, x, x_hat, x.copy(), 0.01, pt, ee, lam, 1e4, 1e-3, 1e-8, extra)


def medium(seed: int = 2, nx: int = 4, ny: int = 5, n: int = 10, n_pt: int = 12000, n_ee: int = 8000):
    """A 4x5 array of rotated unit cubes (10^3 cells each) packed with small gaps."""
    a = 1.0 / n
    base, btets = kuhn_cube(n, a)
    bfaces = boundary_faces(btets)
    rots = cube_rotations()
    rr = _rng(seed, "rotation").integers(0, 24, size=nx * ny)
    gx = _rng(seed, "gaps").uniform(1e-5, 1e-3, size=nx - 1)
    gy = _rng(seed, "gaps-y").uniform(1e-5, 1e-3, size=ny - 1)
    ox = np.concatenate([[0.0], np.cumsum(1.0 + gx)])
    oy = np.concatenate([[0.0], np.cumsum(1.0 + gy)])
    Ecube = _rng(seed, "material").uniform(1e4, 1e6, size=nx * ny)
    nb = len(base)
    rest, x, tets, E = [], [], [], []
    cubes = {}
    for iy in range(ny):
        for ix in range(nx):
            c = iy * nx + ix
            R = rots[rr[c]].astype(np.float64)
            off = c * nb
            rest.append(base)
            # rotate the cube about its centre, then translate into the array
            xc = (base - 0.5) @ R.T + 0.5 + np.array([ox[ix], oy[iy], 0.0])
            x.append(xc)
            tets.append(btets + off)
            E.append(np.full(len(btets), Ecube[c]))
            cubes[(ix, iy)] = (off, xc)
    rest = np.concatenate(rest)
    x = np.concatenate(x)
    tets = np.concatenate(tets)
    E = np.concatenate(E)
    N, T = len(rest), len(tets)
    interfaces = []
    for iy in range(ny):
        for ix in range(nx):
            off, xc = cubes[(ix, iy)]
            f = bfaces + off
            if ix + 1 < nx:
                off2, _ = cubes[(ix + 1, iy)]
                a_side = _Surface(_face_on_plane(f, x, 0, ox[ix] + 1.0))
                b_side = _Surface(_face_on_plane(bfaces + off2, x, 0, ox[ix + 1]))
                interfaces.append((a_side, b_side))
            if iy + 1 < ny:
                off2, _ = cubes[(ix, iy + 1)]
                a_side = _Surface(_face_on_plane(f, x, 1, oy[iy] + 1.0))
                b_side = _Surface(_face_on_plane(bfaces + off2, x, 1, oy[iy + 1]))
                interfaces.append((a_side, b_side))
    fixed = np.zeros(N, dtype=np.uint8)
    x_hat = x + _rng(seed, "noise").normal(0.0, 0.01 * a, size=(N, 3))
    pt, ee = _pick(x, interfaces, n_pt, n_ee)
    lam = np.exp(_rng(seed, "lambda").uniform(np.log(1.0), np.log(1e3), size=len(pt) + len(ee)))
    return _finish("medium", seed, rest, tets, E, np.full(T, 0.45), np.full(T, 1000.0), fixed,
                   x, x_hat, x.copy(), 0.01, pt, ee, lam, 1e4, 1e-3, 1e-5)


def large(seed: int = 3, nxy: int = 50, nz: int = 30, blocks: int = 5, a: float = 0.02,
          n_pt: int = 600000, n_ee: int = 400000):
    """Five 50x50x30-cell blocks stacked in z, compressed by 40 % between fixed planes."""
    # one block: nxy x nxy x nz cells at spacing a
    base, btets = kuhn_box(nxy, nxy, nz, a)
    bfaces = boundary_faces(btets)
    nb = len(base)
    h_block = nz * a
    gap = 1e-3
    scale = 0.6
    rest, tets, x = [], [], []
    tops, bots = [], []
    for b in range(blocks):
        off = b * nb
        zo = b * (h_block + gap)
        rb = base + np.array([0.0, 0.0, zo])
        rest.append(rb)
        xb = rb.copy()
        xb[:, 2] *= scale
        x.append(xb)
        tets.append(btets + off)
        tops.append(_Surface(_face_on_plane(bfaces, base, 2, h_block) + off))
        bots.append(_Surface(_face_on_plane(bfaces, base, 2, 0.0) + off))
    rest = np.concatenate(rest)
    x = np.concatenate(x)
    tets = np.concatenate(tets)
    N, T = len(rest), len(tets)
    fixed = np.zeros(N, dtype=np.uint8)
    fixed[:nb][base[:, 2] == 0.0] = 1
    fixed[(blocks - 1) * nb:][base[:, 2] == h_block] = 1
    sigma = 0.01 * a * scale
    x_hat = x + _rng(seed, "noise").normal(0.0, sigma, size=(N, 3)) * (1 - fixed)[:, None]
    interfaces = [(tops[b], bots[b + 1]) for b in range(blocks - 1)]
    pt, ee = _pick(x, interfaces, n_pt, n_ee)
    lam = np.exp(_rng(seed, "lambda").uniform(np.log(1.0), np.log(1e4), size=len(pt) + len(ee)))
    return _finish("large", seed, rest, tets, np.full(T, 1e5), np.full(T, 0.4), np.full(T, 1000.0),
                   fixed, x, x_hat, x.copy(), 0.01, pt, ee, lam, 1e5, 1e-3, 1e-5)


def bar(nx: int = 8, n: int = 2, a: float = 0.1, stretch: float = 1.1, dt: float = 100.0):
    """A bar of nx x n x n cells (spacing a) along x, E = 1e4, nu = 0, rho = 1000;
    both end faces are moving-boundary nodes, the far one (x = nx a) moved to
    stretch * nx a in x_hat^[0]; x = x_tilde = rest, no constraints.  With
    nu = 0 the static solution is the homogeneous stretch (stretch X, Y, Z),
    and with dt = 100 s the inertia term is ~1e-7 of the elastic one."""
    rest, tets = kuhn_box(nx, n, n, a)
    N, T = len(rest), len(tets)
    L = nx * a
    fixed = ((np.abs(rest[:, 0]) < 1e-12) | (np.abs(rest[:, 0] - L) < 1e-12)).astype(np.uint8)
    x = rest.copy()
    x_hat = x.copy()
    far = np.abs(rest[:, 0] - L) < 1e-12
    x_hat[far, 0] = stretch * L
    return _finish("bar", 0, rest, tets, np.full(T, 1e4), np.zeros(T), np.full(T, 1000.0), fixed, x, x_hat,
                   x.copy(), dt, np.zeros((0, 4)), np.zeros((0, 4)), np.zeros(0), 1e4, 1e-3, 1e-8)


def falling_cubes(v: float = -0.5, dt: float = 0.01, n: int = 4, lateral=(0.37, 0.21), jitter: float = 0.0,
                  seed: int = 6):
    """The two-cube stack (1 mm gap, bottom face of the lower cube fixed) with
    the upper cube moving down at v m/s: x_tilde = x + dt v on its nodes, so
    one step of 5 mm would cross the gap; x_hat^[0] = x; no constraints yet.
    jitter > 0 moves every free node of x by N(0, jitter) first, so that no two
    contact pairs are tied in collision time."""
    a, rest, tets, n_lo, top, bot, _ = _stack_two_cubes(n, 1e-3, lateral)
    N, T = len(rest), len(tets)
    fixed = np.zeros(N, dtype=np.uint8)
    fixed[:n_lo][rest[:n_lo, 2] == 0.0] = 1
    x = rest.copy()
    if jitter > 0.0:
        x += _rng(seed, "jitter").normal(0.0, jitter, size=x.shape) * (1 - fixed)[:, None]
    xt = x.copy()
    xt[n_lo:, 2] += dt * v
    return _finish("falling_cubes", 0, rest, tets, np.full(T, 1e5), np.full(T, 0.4), np.full(T, 1000.0), fixed, x,
                   x.copy(), xt, dt, np.zeros((0, 4)), np.zeros((0, 4)), np.zeros(0), 1e4, 1e-3, 1e-8)


def slope(n: int = 4, E: float = 1e7, incline: float = float(np.arctan(0.5)), dt: float = 0.01):
    """The two-cube stack with the lower cube fixed (the ground) and the upper
    one resting 1 mm above it, under gravity tilted by `incline` (the same as
    an inclined ground: g = 9.8 (sin, 0, -cos)), stiff enough (E = 1e7) to
    slide as a body.  x_tilde is left to the caller, who adds h v + h^2 g per
    step; scene["gravity"] holds g."""
    sc = dict(falling_cubes(v=0.0, dt=dt, n=n))
    N, T = len(sc["x"]), len(sc["tets"])
    fixed = sc["fixed"].copy()
    fixed[: N // 2] = 1
    sc["fixed"] = fixed
    sc["E"] = np.full(T, E)
    sc["gravity"] = 9.8 * np.array([np.sin(incline), 0.0, -np.cos(incline)])
    sc["name"] = "slope"
    return sc


def ccd_target(sc: dict, recipe: str, seed: int = 11) -> np.ndarray:
    """A target state x_hat for the collision queries along x -> x_hat.

    push       the upper cube of a two-cube stack (rest z > 1) 4 mm down into
               the lower one, every free node jittered by N(0, 0.5 mm);
    push_deep  the same, 0.3 down (through more than one cell layer), jitter 5 mm;
    jitter     every free node moved by N(0, 0.3 mm) (the cubes' gaps are 0.01-1 mm);
    layers     block b of the stacked blocks (rest z in [0.601 b, 0.601 b + 0.6])
               1 mm * b down, so each interface (gap 0.6 mm) interpenetrates by
               0.4 mm, jitter N(0, 0.1 mm);
    static     x_hat = x.
    Fixed nodes stay at x."""
    rng = _rng(seed, "ccd_" + recipe)
    x = sc["x"]
    rest = sc["rest"]
    xh = x.copy()
    if recipe == "push":
        xh += rng.normal(0.0, 5e-4, size=x.shape)
        xh[rest[:, 2] > 1.0, 2] -= 0.004
    elif recipe == "push_deep":
        xh += rng.normal(0.0, 5e-3, size=x.shape)
        xh[rest[:, 2] > 1.0, 2] -= 0.3
    elif recipe == "jitter":
        xh += rng.normal(0.0, 3e-4, size=x.shape)
    elif recipe == "layers":
        b = np.floor(rest[:, 2] / 0.601 + 1e-9)
        xh += rng.normal(0.0, 1e-4, size=x.shape)
        xh[:, 2] -= 1e-3 * b
    elif recipe != "static":
        raise ValueError(recipe)
    fixed = sc["fixed"].astype(bool)
    xh[fixed] = x[fixed]
    return xh


def serve_request(i: int):
    """One request of the serving stream: two stacked n^3 cubes, tets ~ LogU[2k, 300k]."""
    r = _rng(1000 + i, "size")
    T_target = np.exp(r.uniform(np.log(2e3), np.log(3e5)))
    n = int(np.clip(np.rint(np.cbrt(T_target / 12.0)), 6, 29))
    a, rest, tets, n_lo, top, bot, n_surf = _stack_two_cubes(n, 1e-3)
    N, T = len(rest), len(tets)
    fixed = np.zeros(N, dtype=np.uint8)
    fixed[:n_lo][rest[:n_lo, 2] == 0.0] = 1
    x = rest.copy()
    x_hat = x + _rng(1000 + i, "noise").normal(0.0, 0.01 * a, size=(N, 3)) * (1 - fixed)[:, None]
    n_c = int(round(0.4 * n_surf))
    n_pt = int(round(0.6 * n_c))
    n_ee = n_c - n_pt
    pt, ee = _pick(x, [(top, bot)], n_pt, n_ee)
    lam = np.exp(_rng(1000 + i, "lambda").uniform(0.0, np.log(1e3), size=n_c))
    return _finish(f"serve{i}", 1000 + i, rest, tets, np.full(T, 1e5), np.full(T, 0.4),
                   np.full(T, 1000.0), fixed, x, x_hat, x.copy(), 0.01, pt, ee, lam, 1e4, 1e-3, 1e-5)


def make_scene(name: str, seed: int | None = None, **kw):
    builders = {"tiny": (tiny, 1), "medium": (medium, 2), "large": (large, 3)}
    fn, s = builders[name]
    return fn(s if seed is None else seed, **kw)
