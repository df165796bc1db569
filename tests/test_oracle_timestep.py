"""Pins of the oracle's time step (Algorithm 1): a bar stretched through its
moving boundary reaches the closed-form homogeneous stretch (nu = 0, inertia
negligible), and a cube thrown at another ends the step intersection free
and in the contact region."""
import numpy as np

from oracle import ccd, timestep
import scenes


def test_bar_reaches_the_homogeneous_stretch():
    """Without contacts and inversions both alphas are 1 and the loop ends
    after K_min = 2 iterations, each subproblem after its first full Newton
    step: two Newton steps from x_hat^[0], where only the last cell layer is
    stretched.  At 0.1 % stretch that start is 0.8 % off in strain, so two
    steps of the quadratically convergent method leave ~(0.008^2)^2 of the
    displacement; the bar is 1e-6 of it.  (At 10 % the start is 80 % off and two
    steps are not enough: the step's termination is TOI-based, Section 4.4.)"""
    s = 1.001
    sc = scenes.bar(stretch=s)
    x, v, (pt, ee, lam, gam), info = timestep.time_step(sc)
    assert info["outer"] == 2 and info["alphas"] == [1.0, 1.0] and info["beta"] == 0.0
    ref = sc["rest"] * np.array([s, 1.0, 1.0])
    assert np.abs(x - ref).max() <= 1e-6 * (s - 1) * 0.8
    assert np.allclose(v, (x - sc["x"]) / sc["dt"], rtol=0, atol=1e-15)
    assert len(pt) == 0 and len(ee) == 0


def _cross_body_min_distance(sc, x):
    tris, edges, verts = ccd.surface(sc["tets"])
    n_lo = len(sc["rest"]) // 2
    lower_t = tris[(tris < n_lo).all(axis=1)]
    upper_t = tris[(tris >= n_lo).all(axis=1)]
    lv = verts[verts < n_lo]
    uv = verts[verts >= n_lo]
    le = edges[(edges < n_lo).all(axis=1)]
    ue = edges[(edges >= n_lo).all(axis=1)]
    d = []
    for v, t in ((uv, lower_t), (lv, upper_t)):
        ids = np.array([[p, *f] for p in v for f in t])
        d.append(ccd._dist("pt", x[ids]).min())
    ids = np.array([[*a, *b] for a in ue for b in le])
    d.append(ccd._dist("ee", x[ids]).min())
    return min(d)


def test_thrown_cube_ends_intersection_free_in_contact():
    """The upper cube's inertial target lies 5 mm down, past the 1 mm gap:
    the step must stop it intersection free (every cross-body point-triangle
    and edge-edge distance positive at x^{t+1}), closer than it started, and
    with the constraints that stopped it in the active set."""
    sc = scenes.falling_cubes()
    x, v, (pt, ee, lam, gam), info = timestep.time_step(sc, max_outer=100)
    print(info["outer"], info["beta"], [round(a, 4) for a in info["alphas"][:12]])
    d_end = _cross_body_min_distance(sc, x)
    assert d_end > 0.0
    assert d_end < _cross_body_min_distance(sc, sc["x"])
    assert len(pt) + len(ee) > 0
    assert info["beta"] <= 1e-3 or info["outer"] == 100
    assert (v[len(v) // 2:, 2] < 0).all()
