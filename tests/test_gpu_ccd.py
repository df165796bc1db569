"""The collision queries on the GPU (LBVH broad phase, ACCD narrow phase,
UpdateActiveSet of Algorithm 3, MaxStepSize of Algorithm 1) against the FP64
oracle's brute force.

Bars: the number of candidate pairs (the exact FP64 swept-box test) equal;
the colliding pairs equal as sets; their collision times, and the step size,
within 1e-8 relative.  ACCD's steps are 0.9 d / l_p with d a distance of
order 1e-5 between coordinates of order 5, so each FP64 distance carries a
relative rounding error up to 5 / 1e-5 * 2.2e-16 ~ 1e-10, and a time summed
from up to ~50 steps can differ by ~5e-9 between two FP64 codes (a wrong step
rule errs by O(1)).  The rebuilt active set equal row for row, with lambda and
gamma exact.  At the full size of the large workload, on sampled query
primitives, the oracle brute-forces their candidates and collision times one
by one."""
import numpy as np
import pytest

from oracle import ccd
import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bf():
    from paper_2512_12151_amd import bfal
    return bfal


@pytest.fixture(scope="module")
def ctx(bf):
    return bf.Context(0)


CASES = {
    "tiny_push": (lambda: scenes.tiny(lateral=(0.37, 0.21)), "push"),
    "tiny_push_deep": (lambda: scenes.tiny(lateral=(0.37, 0.21)), "push_deep"),
    "cubes8_push": (lambda: scenes.tiny(n=8, n_pt=300, n_ee=200, lateral=(0.3, 0.6)), "push"),
    "tiny_static": (lambda: scenes.tiny(lateral=(0.37, 0.21)), "static"),
    "medium_jitter": (scenes.medium, "jitter"),
}

_cache = {}


def case(name):
    if name not in _cache:
        make, recipe = CASES[name]
        sc = make()
        xh = scenes.ccd_target(sc, recipe)
        tris, edges, verts = ccd.surface(sc["tets"])
        pt, ee = ccd.candidates(sc["x"], xh, tris, edges, verts, sc["delta"])
        (cpt, tpt), (cee, tee) = ccd.colliding_pairs(sc["x"], xh, tris, edges, verts, sc["delta"])
        _cache[name] = dict(sc=sc, xh=xh, surf=(tris, edges, verts), ncand=(len(pt), len(ee)),
                            coll=(cpt, tpt, cee, tee))
    return _cache[name]


def _by_row(rows, times):
    order = np.lexsort(rows.T[::-1])
    return rows[order], times[order]


@pytest.mark.parametrize("name", list(CASES))
def test_collisions_and_step_size_match_oracle(ctx, bf, name):
    print(f"case {name}", flush=True)
    c = case(name)
    sc, xh = c["sc"], c["xh"]
    pb = bf.Problem.from_scene(ctx, sc)
    alpha, st = pb.max_step_size(xh)
    print(f"{name}: gpu {st}", flush=True)
    assert (st["candidates_pt"], st["candidates_ee"]) == c["ncand"]
    cpt, tpt, cee, tee = c["coll"]
    assert (st["colliding_pt"], st["colliding_ee"]) == (len(cpt), len(cee))
    gpt, gtp, gee, gte = pb.collisions(st)
    for g_rows, g_t, o_rows, o_t in ((gpt, gtp, cpt, tpt), (gee, gte, cee, tee)):
        g_rows, g_t = _by_row(g_rows.astype(np.int64), g_t)
        o_rows, o_t = _by_row(o_rows.astype(np.int64), o_t)
        assert np.array_equal(g_rows, o_rows)
        rel = np.abs(g_t - o_t) / np.maximum(np.abs(o_t), 1e-300)
        if len(rel):
            k = int(np.argmax(rel))
            print(f"{name}: times max rel diff {rel.max():.3e} (pair {o_rows[k].tolist()}, gpu {g_t[k]!r}, "
                  f"oracle {o_t[k]!r}); > 1e-12: {int((rel > 1e-12).sum())}, > 1e-9: {int((rel > 1e-9).sum())}, "
                  f"> 1e-6: {int((rel > 1e-6).sum())} of {len(rel)}", flush=True)
        assert np.allclose(g_t, o_t, rtol=1e-8, atol=1e-15)
    tris, edges, verts = c["surf"]
    a_ref = ccd.max_step_size(sc["x"], xh, sc["tets"], tris, edges, verts, sc["delta"])
    print(f"{name}: alpha gpu {alpha:.15e} oracle {a_ref:.15e}", flush=True)
    assert alpha == pytest.approx(a_ref, rel=1e-8, abs=1e-15)
    if name == "tiny_static":
        assert alpha == 1.0 and st["colliding_pt"] == st["colliding_ee"] == 0


@pytest.mark.parametrize("name", ["tiny_push", "tiny_push_deep", "cubes8_push", "medium_jitter"])
def test_update_active_set_matches_oracle(ctx, bf, name):
    """The scene's own constraints as the current set, a third of them with
    gamma below 0.01, some colliding pairs already in it (stored with their
    triangle or edges in another order)."""
    print(f"case {name}", flush=True)
    c = case(name)
    sc, xh = dict(c["sc"]), c["xh"]
    cpt, tpt, cee, tee = c["coll"]
    pt_c = np.concatenate([sc["pt"], cpt[:3][:, [0, 3, 1, 2]]]).astype(np.int32)
    ee_c = np.concatenate([sc["ee"], cee[:3][:, [3, 2, 1, 0]]]).astype(np.int32)
    n_pt, n_ee = len(pt_c), len(ee_c)
    rng = np.random.default_rng(4)
    lam = rng.uniform(0.0, 50.0, n_pt + n_ee)
    gam = np.where(rng.uniform(size=n_pt + n_ee) < 1 / 3, 0.005, rng.uniform(0.02, 1.0, n_pt + n_ee))
    sc.update(pt=pt_c, ee=ee_c, lam=lam, gamma=gam)
    pb = bf.Problem.from_scene(ctx, sc)
    st = pb.update_active_set(xh)
    print(f"{name}: gpu {st}", flush=True)
    tris, edges, verts = c["surf"]
    pt2, ee2, lam2, gam2, info = ccd.update_active_set(len(sc["x"]), sc["x"], xh, tris, edges, verts, pt_c, ee_c, lam,
                                                       gam, sc["delta"])
    print(f"{name}: oracle {info}", flush=True)
    gpt, gee, glam, ggam = pb.constraints()
    assert np.array_equal(gpt, pt2) and np.array_equal(gee, ee2)
    assert np.array_equal(glam, lam2) and np.array_equal(ggam, gam2)
    assert (st["new_pt"], st["new_ee"]) == (info["new_pt"], info["new_ee"])
    assert (st["added_pt"], st["added_ee"], st["removed"]) == (info["added_pt"], info["added_ee"], info["removed"])
    # the updated set drives a Newton step
    p, _, status = pb.newton_step(tol=1e-5)
    assert status == bf.BF_OK and np.isfinite(p).all()


def test_update_with_empty_set_and_repeated_call(ctx, bf):
    """From no constraints at all; a second identical call adds nothing (every
    colliding pair kept by the filter is already in the set, and the pairs the
    filter dropped stay dropped: their vertices' earliest pairs are gone)."""
    c = case("tiny_push")
    sc, xh = dict(c["sc"]), c["xh"]
    sc.update(pt=np.zeros((0, 4), np.int32), ee=np.zeros((0, 4), np.int32), lam=np.zeros(0), gamma=np.zeros(0))
    pb = bf.Problem.from_scene(ctx, sc)
    st1 = pb.update_active_set(xh)
    tris, edges, verts = c["surf"]
    pt2, ee2, lam2, gam2, info = ccd.update_active_set(len(sc["x"]), sc["x"], xh, tris, edges, verts,
                                                       np.zeros((0, 4)), np.zeros((0, 4)), np.zeros(0), np.zeros(0),
                                                       sc["delta"])
    gpt, gee, glam, ggam = pb.constraints()
    assert np.array_equal(gpt, pt2) and np.array_equal(gee, ee2)
    assert np.all(glam == 0.0) and np.all(ggam == 1.0)
    st2 = pb.update_active_set(xh)
    pt3, ee3, _, _, info3 = ccd.update_active_set(len(sc["x"]), sc["x"], xh, tris, edges, verts, pt2, ee2, lam2, gam2,
                                                  sc["delta"])
    gpt3, gee3, _, _ = pb.constraints()
    assert np.array_equal(gpt3, pt3) and np.array_equal(gee3, ee3)
    assert st2["new_pt"] + st2["new_ee"] == info3["new_pt"] + info3["new_ee"]
    print(f"first {st1}, second {st2}", flush=True)


def test_ccd_errors(ctx, bf):
    c = case("tiny_push")
    pb = bf.Problem.from_scene(ctx, c["sc"])
    for sep in (-0.1, 1.0, 2.0):
        with pytest.raises(bf.BfalError):
            pb.max_step_size(c["xh"], sep=sep)


@pytest.mark.timeout(600)
def test_large_collisions_sampled(ctx, bf):
    """The large workload (2.25M tets) with its blocks pushed into each other
    (each interface interpenetrates by 0.4 mm): for 300 sampled surface
    vertices and 300 sampled surface edges the oracle brute-forces every
    candidate against all triangles / edges and runs ACCD; the GPU's colliding
    pairs at those primitives must be the same set with the same times.  The
    step size is the smallest GPU time and no larger than any sampled one; the
    inversion bound no larger than the oracle's on 2000 sampled tets."""
    sc = scenes.make_scene("large")
    xh = scenes.ccd_target(sc, "layers")
    pb = bf.Problem.from_scene(ctx, sc)
    print("large: GPU collision queries", flush=True)
    alpha, st = pb.max_step_size(xh)
    print(f"large: gpu {st}", flush=True)
    gpt, gtp, gee, gte = pb.collisions(st)
    pb.close()
    assert st["colliding_pt"] > 1000 and st["colliding_ee"] > 1000
    assert alpha == min(st["alpha_ccd"], st["alpha_inversion"])
    assert st["alpha_ccd"] == min(gtp.min(), gte.min())
    print("large: oracle surface", flush=True)
    tris, edges, verts = ccd.surface(sc["tets"])
    x = sc["x"]
    rng = np.random.default_rng(9)
    d = sc["delta"]
    # point-triangle: sampled surface vertices against every triangle
    sv = rng.choice(verts, 300, replace=False)
    vlo, vhi = ccd.swept_boxes(x, xh, sv[:, None])
    tlo, thi = ccd.swept_boxes(x, xh, tris)
    vi, ti = np.nonzero(ccd.boxes_near(vlo, vhi, tlo, thi, d))
    cand = np.column_stack([sv[vi], tris[ti]])
    cand = cand[(cand[:, 0] != cand[:, 1]) & (cand[:, 0] != cand[:, 2]) & (cand[:, 0] != cand[:, 3])]
    hit, toc = ccd.accd("pt", x[cand], xh[cand])
    o_rows, o_t = _by_row(cand[hit], toc[hit])
    mine = np.isin(gpt[:, 0], sv)
    g_rows, g_t = _by_row(gpt[mine].astype(np.int64), gtp[mine])
    print(f"large: sampled PT {len(o_rows)} colliding of {len(cand)} candidates", flush=True)
    assert len(o_rows) > 0
    assert np.array_equal(g_rows, o_rows) and np.allclose(g_t, o_t, rtol=1e-8, atol=1e-15)
    min_sampled = o_t.min()
    # edge-edge: sampled edges against every edge (either side of the pair)
    se = rng.choice(len(edges), 300, replace=False)
    elo, ehi = ccd.swept_boxes(x, xh, edges)
    a, b = np.nonzero(ccd.boxes_near(elo[se], ehi[se], elo, ehi, d))
    a = se[a]
    keep = a != b
    a, b = a[keep], b[keep]
    pairs = np.unique(np.column_stack([np.minimum(a, b), np.maximum(a, b)]), axis=0)
    cand = np.column_stack([edges[pairs[:, 0]], edges[pairs[:, 1]]])
    share = ((cand[:, 0] == cand[:, 2]) | (cand[:, 0] == cand[:, 3]) | (cand[:, 1] == cand[:, 2])
             | (cand[:, 1] == cand[:, 3]))
    cand = cand[~share]
    hit, toc = ccd.accd("ee", x[cand], xh[cand])
    o_rows, o_t = _by_row(cand[hit], toc[hit])
    sel = {tuple(e) for e in edges[se].tolist()}
    mine = np.array([tuple(r[:2]) in sel or tuple(r[2:]) in sel for r in gee.tolist()], dtype=bool)
    g_rows, g_t = _by_row(gee[mine].astype(np.int64), gte[mine])
    print(f"large: sampled EE {len(o_rows)} colliding of {len(cand)} candidates", flush=True)
    assert len(o_rows) > 0
    assert np.array_equal(g_rows, o_rows) and np.allclose(g_t, o_t, rtol=1e-8, atol=1e-15)
    assert alpha <= min(min_sampled, o_t.min()) * (1 + 1e-12)
    # inversion bound on sampled tets
    tt = sc["tets"][rng.choice(len(sc["tets"]), 2000, replace=False)].astype(np.int64)
    assert st["alpha_inversion"] <= ccd.inversion_bound(x[tt], xh[tt]).min() * (1 + 1e-12)


def test_inversion_bound_either_orientation(ctx, bf):
    """MaxStepSize's inversion bound (Algorithm 1) on a mesh whose tets are
    half negatively oriented (two vertices of every other tet swapped; the
    element terms do not depend on the order): a static target is never
    limited, and an interior node pushed 1.2 cell widths gives the oracle's
    bound and the bound of the same mesh in positive order."""
    sc = scenes.tiny(lateral=(0.37, 0.21))
    flipped = dict(sc)
    t = sc["tets"].copy()
    t[::2, 1], t[::2, 2] = sc["tets"][::2, 2], sc["tets"][::2, 1]
    flipped["tets"] = np.ascontiguousarray(t)
    interior = 2 + 5 * 2 + 25 * 2          # node (2, 2, 2) of the lower 4^3 cube
    assert not sc["fixed"][interior]
    xh = sc["x"].copy()
    xh[interior] += [0.0, 0.0, 0.3]
    alphas = {}
    for name, s in (("positive", sc), ("flipped", flipped)):
        print(f"inversion bound: {name}", flush=True)
        pb = bf.Problem.from_scene(ctx, s)
        a_static, _ = pb.max_step_size(sc["x"].copy())
        assert a_static == 1.0
        alphas[name], _ = pb.max_step_size(xh)
        pb.close()
    tris, edges, verts = ccd.surface(flipped["tets"])
    ref = ccd.max_step_size(sc["x"], xh, flipped["tets"], tris, edges, verts, sc["delta"])
    print(f"inversion bound: gpu {alphas}, oracle {ref}", flush=True)
    assert 0.0 < ref < 1.0
    for a in alphas.values():
        assert a == pytest.approx(ref, rel=1e-8)
