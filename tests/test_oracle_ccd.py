"""Pins of the oracle's collision side (UpdateActiveSet, Algorithm 3, and
MaxStepSize, Algorithm 1): the surface of a Kuhn grid against closed counts,
ACCD against closed-form approach times and against densely sampled
distances of random trajectories, the earliest-time filter on a hand-made
case, the active-set bookkeeping, and the inversion bound against closed
forms."""
import numpy as np
import pytest

from oracle import ccd, core
import scenes
from scenes import mesh

RNG = np.random.default_rng(7)
S = ccd.S_SEP


def kuhn_cube(n):
    rest, tets = mesh.kuhn_cube(n, 1.0 / n)
    return rest, tets


@pytest.mark.parametrize("n", [1, 2, 4])
def test_surface_of_a_kuhn_cube(n):
    rest, tets = kuhn_cube(n)
    tris, edges, verts = ccd.surface(tets)
    # each of the 6 faces has n^2 squares split into 2 triangles
    assert len(tris) == 12 * n * n
    # closed surface of genus 0: E = 3F/2 and V - E + F = 2
    assert len(edges) * 2 == 3 * len(tris)
    assert len(verts) - len(edges) + len(tris) == 2
    # every boundary triangle lies on one face of the cube
    P = rest[tris]
    on_face = np.zeros(len(tris), dtype=bool)
    for k in range(3):
        for v in (0.0, 1.0):
            on_face |= np.all(np.abs(P[:, :, k] - v) < 1e-12, axis=1)
    assert on_face.all()
    # the surface vertices are exactly the grid nodes on the boundary
    on_bnd = np.any((np.abs(rest) < 1e-12) | (np.abs(rest - 1.0) < 1e-12), axis=1)
    assert np.array_equal(verts, np.nonzero(on_bnd)[0])


def _pt_approach(d0, v, lateral=(0.2, 0.3)):
    """A point above the interior of a static triangle in z = 0 moving down
    at speed v over t in [0, 1]."""
    tri = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])
    p0 = np.array([lateral[0], lateral[1], d0])
    X0 = np.vstack([p0, tri])[None]
    X1 = X0.copy()
    X1[0, 0, 2] -= v
    return X0, X1


@pytest.mark.parametrize("d0,v", [(1e-3, 2e-3), (0.05, 0.5), (0.3, 0.31)])
def test_accd_point_triangle_closed_form(d0, v):
    """d(t) = d0 - v t, l_p = v: the first step lands exactly on the gap s d0,
    the second below it, so toc = (1 - s) d0 / v = (1 - s) t* with t* = d0/v."""
    X0, X1 = _pt_approach(d0, v)
    hit, toc = ccd.accd("pt", X0, X1)
    assert hit[0]
    assert toc[0] == pytest.approx((1 - S) * d0 / v, rel=1e-12)
    # a common translation of all four vertices changes nothing
    shift = np.array([0.3, -0.7, 0.11])
    hit2, toc2 = ccd.accd("pt", X0 + shift, X1 + 2 * shift)
    assert hit2[0] and toc2[0] == pytest.approx(toc[0], rel=1e-12)


def test_accd_point_triangle_misses():
    X0, X1 = _pt_approach(0.1, 0.05)         # stops at half the gap
    hit, toc = ccd.accd("pt", X0, X1)
    assert not hit[0] and toc[0] == 1.0
    X0, X1 = _pt_approach(0.1, 0.5, lateral=(2.0, 2.0))   # passes beside the triangle
    hit, _ = ccd.accd("pt", X0, X1)
    assert not hit[0]


def test_accd_edge_edge_closed_form():
    """Perpendicular skew edges, the upper one moving down along the common
    perpendicular: d(t) = d0 - v t with l_p = v, so toc = (1 - s) d0 / v."""
    d0, v = 0.02, 0.05
    a0, a1 = np.array([-1.0, 0.0, d0]), np.array([1.0, 0.0, d0])
    b0, b1 = np.array([0.0, -1.0, 0.0]), np.array([0.0, 1.0, 0.0])
    X0 = np.array([[a0, a1, b0, b1]])
    X1 = X0.copy()
    X1[0, :2, 2] -= v
    hit, toc = ccd.accd("ee", X0, X1)
    assert hit[0] and toc[0] == pytest.approx((1 - S) * d0 / v, rel=1e-12)


def _sampled(kind, X0, X1, ns=2001):
    ts = np.linspace(0.0, 1.0, ns)
    d = np.stack([ccd._dist(kind, X0 + t * (X1 - X0)) for t in ts], axis=1)
    return ts, d


@pytest.mark.parametrize("kind", ["pt", "ee"])
def test_accd_is_conservative_on_random_trajectories(kind):
    """Between two ACCD iterates the distance can shrink by at most l_p times
    the step, so d(t) >= 0.1 d_i on every step; hence before toc the sampled
    distance stays above 0.1 s d0 > 0, a pair that intersects somewhere in
    [0, 1] is reported with toc before that time, and a pair reported as
    missing stays above 0.1 s d0 over the whole path."""
    n = 400
    X0 = RNG.uniform(-1, 1, (n, 4, 3))
    # move the primitives toward each other by random amounts
    c = X0.mean(axis=1, keepdims=True)
    disp = RNG.normal(0, 0.6, (n, 4, 3))
    disp[:, :2 if kind == "ee" else 1] += -0.8 * (X0[:, :2 if kind == "ee" else 1] - c)
    X1 = X0 + disp
    hit, toc = ccd.accd(kind, X0, X1)
    ts, d = _sampled(kind, X0, X1)
    d0 = d[:, 0]
    assert hit.any() and (~hit).any()
    for i in range(n):
        if hit[i]:
            before = ts <= toc[i]
            assert d[i, before].min() >= 0.1 * S * d0[i] * (1 - 1e-9)
        else:
            assert d[i].min() >= 0.1 * S * d0[i] * (1 - 1e-9)
        crossing = np.nonzero(d[i] <= 1e-9 * d0[i])[0]
        if len(crossing):
            assert hit[i] and toc[i] <= ts[crossing[0]]


def test_earliest_filter_hand_case():
    """Pairs A (verts 0,1,2,3; T=0.5), B (0,4,5,6; T=0.2), C (7,8,9,10; T=0.9)
    and the edge pair D (1,7,11,12; T=0.6): A is vertex 1's earliest, B vertex
    0's, C vertex 8's, D vertex 11's -- all survive.  Then C moves to T=0.95, a
    pair E on C's vertices comes at T=0.1, and D becomes (1,7,2,3): C is no
    vertex's earliest (E is), nor is D (A holds 1, 2, 3 at 0.5, E holds 7)."""
    pt = np.array([[0, 1, 2, 3], [0, 4, 5, 6], [7, 8, 9, 10]])
    ee = np.array([[1, 7, 11, 12]])
    kpt, kee = ccd.earliest_filter(13, pt, np.array([0.5, 0.2, 0.9]), ee, np.array([0.6]))
    assert kpt.all() and kee.all()
    pt2 = np.array([[0, 1, 2, 3], [0, 4, 5, 6], [7, 8, 9, 10], [7, 8, 9, 10]])
    ee2 = np.array([[1, 7, 2, 3]])
    kpt, kee = ccd.earliest_filter(13, pt2, np.array([0.5, 0.2, 0.95, 0.1]), ee2, np.array([0.6]))
    assert list(kpt) == [True, True, False, True] and list(kee) == [False]


def pushed_state(sc, depth=0.004, noise=0.0005, seed=3):
    """x_hat: the upper cube pushed down into the lower one, every free node
    jittered (so the pairs' collision times differ)."""
    rng = np.random.default_rng(seed)
    xh = sc["x"] + noise * rng.standard_normal(sc["x"].shape)
    xh[sc["rest"][:, 2] > 1.0, 2] -= depth
    return np.where(sc["fixed"][:, None] == 1, sc["x"], xh)


def test_earliest_filter_keeps_ties_up_to_rounding():
    """Two pairs at one vertex whose times differ only by rounding are both
    its earliest; a pair 1e-6 later is not."""
    pt = np.array([[0, 1, 2, 3], [0, 4, 5, 6], [0, 7, 8, 9]])
    T = np.array([0.5, 0.5 * (1 + 1e-12), 0.5 * (1 + 1e-6)])
    pt[1:, 1:] = [[1, 2, 3], [1, 2, 3]]            # the later pairs share all of A's vertices
    kpt, _ = ccd.earliest_filter(10, pt, T, np.zeros((0, 4), np.int64), np.zeros(0))
    assert list(kpt) == [True, True, False]


def test_update_active_set_bookkeeping():
    """Two stacked cubes, the upper one pushed into the lower: new pairs enter
    with lambda 0, gamma 1; a pair already in the set is not added again; a
    constraint with gamma below 0.01 is removed; a kept one keeps its values."""
    sc = scenes.tiny(lateral=(0.37, 0.21))
    x = sc["x"]
    xh = pushed_state(sc)
    tris, edges, verts = ccd.surface(sc["tets"])
    (cpt, tpt), (cee, tee) = ccd.colliding_pairs(x, xh, tris, edges, verts, sc["delta"])
    assert len(cpt) > 0 and len(cee) > 0
    # current set: one of the colliding PT pairs (triangle reversed), one EE pair with gamma 0.005
    pt_c = np.array([cpt[0][[0, 3, 2, 1]]])
    ee_c = np.array([cee[0]])
    lam = np.array([3.0, 4.0])
    gam = np.array([0.5, 0.005])
    pt2, ee2, lam2, gam2, info = ccd.update_active_set(len(x), x, xh, tris, edges, verts, pt_c, ee_c, lam, gam,
                                                       sc["delta"])
    assert np.array_equal(pt2[0], pt_c[0]) and lam2[0] == 3.0 and gam2[0] == 0.5
    keys = {tuple(r) for r in ccd.canonical("pt", pt2)}
    assert len(keys) == len(pt2)                        # no duplicate of the current pair
    assert info["removed"] == 1
    assert not any(np.array_equal(r, ee_c[0]) for r in ee2)   # the decayed EE constraint went
    n_pt = len(pt2)
    assert np.all(lam2[1:n_pt] == 0.0) and np.all(gam2[1:n_pt] == 1.0)
    assert np.all(lam2[n_pt:] == 0.0) and np.all(gam2[n_pt:] == 1.0)
    assert info["added_pt"] == n_pt - 1 and info["added_ee"] == len(ee2)
    assert info["added_pt"] + info["added_ee"] < info["new_pt"] + info["new_ee"]   # the filter dropped some


def test_inversion_bound_closed_forms():
    rest = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    # apex moving through the opposite face: det linear, J(t) = 1 - 2t
    X1 = rest.copy()
    X1[3, 2] = -1.0
    t = ccd.inversion_bound(rest[None], X1[None])
    assert t[0] == pytest.approx((1 - S) / 2, abs=1e-12) and t[0] <= (1 - S) / 2
    # point reflection through the centroid: det(D(t)) = (1 - 2t)^3 det(D(0))
    c = rest.mean(axis=0)
    X1 = 2 * c - rest
    t = ccd.inversion_bound(rest[None], X1[None])
    assert t[0] == pytest.approx((1 - S ** (1 / 3)) / 2, abs=1e-12)
    # no inversion: uniform growth
    t = ccd.inversion_bound(rest[None], 1.5 * rest[None])
    assert t[0] == 1.0


def test_max_step_size_is_the_smallest_bound():
    sc = scenes.tiny(lateral=(0.37, 0.21))
    x = sc["x"]
    xh = pushed_state(sc)
    tris, edges, verts = ccd.surface(sc["tets"])
    a = ccd.max_step_size(x, xh, sc["tets"], tris, edges, verts, sc["delta"])
    (cpt, tpt), (cee, tee) = ccd.colliding_pairs(x, xh, tris, edges, verts, sc["delta"])
    assert a == min(tpt.min(), tee.min())
    assert 0.0 < a < 1.0
    # the state at alpha is intersection free: every candidate pair keeps a positive distance
    xa = x + a * (xh - x)
    pt, ee = ccd.candidates(x, xh, tris, edges, verts, sc["delta"])
    assert ccd._dist("pt", xa[pt]).min() > 0 and ccd._dist("ee", xa[ee]).min() > 0


def test_inversion_bound_does_not_depend_on_vertex_order():
    """A negatively oriented tet (two vertices swapped) gets the bound of the
    same tet in positive order: the closed forms above, and a static tet is
    never limited (before the fix, a negative det D_s(0) gave 0 here)."""
    rest = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    flip = [0, 2, 1, 3]
    X1 = rest.copy()
    X1[3, 2] = -1.0
    t = ccd.inversion_bound(rest[flip][None], X1[flip][None])
    assert t[0] == pytest.approx((1 - S) / 2, abs=1e-12)
    c = rest.mean(axis=0)
    t = ccd.inversion_bound(rest[flip][None], (2 * c - rest)[flip][None])
    assert t[0] == pytest.approx((1 - S ** (1 / 3)) / 2, abs=1e-12)
    assert ccd.inversion_bound(rest[flip][None], rest[flip][None])[0] == 1.0
    assert ccd.inversion_bound(rest[flip][None], 1.5 * rest[flip][None])[0] == 1.0
    # random motions: every tet's bound equals its flipped twin's
    rng = np.random.default_rng(8)
    X0 = rest[None] + rng.normal(0.0, 0.05, size=(50, 4, 3))
    X1 = X0 + rng.normal(0.0, 0.6, size=(50, 4, 3))
    a = ccd.inversion_bound(X0, X1)
    b = ccd.inversion_bound(X0[:, flip], X1[:, flip])
    assert np.allclose(a, b, atol=1e-12) and (a < 1.0).sum() >= 10
