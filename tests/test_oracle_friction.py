"""CPU pins of the friction oracle (Appendix A, IPC's semi-implicit friction)."""
import numpy as np
import pytest

import oracle
from oracle import friction as fr_
import scenes


def test_f0_is_the_norm_above_the_threshold_and_c2_at_it():
    e = 0.3
    y = np.array([0.3, 0.5, 2.0])
    assert np.array_equal(fr_.f0(y, e), y)
    assert np.array_equal(fr_.f1(y, e), np.ones(3))
    assert np.array_equal(fr_.f1_prime(y, e), np.zeros(3))
    below = e * (1 - 1e-9)
    assert fr_.f0(below, e) == pytest.approx(e, abs=1e-9)
    assert fr_.f1(below, e) == pytest.approx(1.0, abs=1e-8)
    assert fr_.f1_prime(below, e) == pytest.approx(0.0, abs=1e-7)
    assert fr_.f0(0.0, e) == pytest.approx(e / 3.0)
    assert fr_.f1(0.0, e) == 0.0
    # f1 and f1' are the derivatives of f0 and f1 (central differences, both branches)
    for yy in (0.01, 0.1, 0.29, 0.31, 1.0):
        hh = 1e-6
        assert (fr_.f0(yy + hh, e) - fr_.f0(yy - hh, e)) / (2 * hh) == pytest.approx(float(fr_.f1(yy, e)), rel=1e-7)
        assert (fr_.f1(yy + hh, e) - fr_.f1(yy - hh, e)) / (2 * hh) == pytest.approx(
            float(fr_.f1_prime(yy, e)), rel=1e-6, abs=1e-7)
    # convex and non-decreasing on [0, inf)
    yy = np.linspace(0, 1, 1001)
    assert np.all(np.diff(fr_.f0(yy, e)) >= 0) and np.all(fr_.f1_prime(yy, e) >= 0)


def test_capture_hand_case():
    """One point 2 mm above the interior of a horizontal triangle: c = d - delta,
    coef = mu_f max(0, lambda - kappa c), normal +z, weights (1, -b0, -b1, -b2)."""
    x = np.array([[0.2, 0.3, 0.002], [0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])
    sc = dict(x=x, dt=0.01, pt=np.array([[0, 1, 2, 3]]), ee=np.zeros((0, 4), dtype=np.int64),
              lam=np.array([30.0]), kappa=1e4, delta=1e-3)
    f = fr_.capture(sc, mu_f=0.4, eps_v=1e-3)
    assert f["coef"][0] == pytest.approx(0.4 * (30.0 - 1e4 * (0.002 - 1e-3)), rel=1e-12)
    assert np.allclose(f["nrm"][0], [0, 0, 1])
    assert np.allclose(f["w"][0], [1.0, -0.5, -0.2, -0.3])
    assert f["e"] == pytest.approx(1e-5)
    sc["lam"] = np.array([5.0])                # lambda < kappa c: no normal force
    assert fr_.capture(sc, 0.4, 1e-3)["coef"][0] == 0.0


def _sliding_scene(seed=1):
    """The shifted tiny stack whose upper cube slides sideways, with a friction
    set captured from its constraints at x (multipliers large enough to press)."""
    sc = dict(scenes.tiny(lateral=(0.37, 0.21)))
    rng = np.random.default_rng(seed)
    sc["lam"] = rng.uniform(20.0, 60.0, size=len(sc["lam"]))
    f = fr_.capture(sc, mu_f=0.5, eps_v=0.5)   # eps_v h = 5 mm: the 1 % noise of x_hat straddles it
    slide = np.zeros_like(sc["x_hat"])
    upper = sc["rest"][:, 2] > 1.0
    # a spread of tangential motions: some contacts stick (|u| < eps_v h), some slide
    slide[upper, 0] = np.linspace(0.0, 3e-4, upper.sum())
    sc["x_hat"] = sc["x_hat"] + slide
    sc["friction"] = f
    return sc, f


def test_friction_gradient_and_hessian_are_derivatives():
    sc, f = _sliding_scene()
    _, y = fr_._tangent(f, sc["x_hat"])
    assert (y < f["e"]).any() and (y > f["e"]).any() and (f["coef"] > 0).all()
    xh = sc["x_hat"]
    G = np.zeros_like(xh)
    rows, cols, vals = [], [], []
    fr_.add_to(f, xh, G, rows, cols, vals)
    import scipy.sparse as sp
    N = len(xh)
    H = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(3 * N, 3 * N)).tocsr()
    rng = np.random.default_rng(3)
    hh = 1e-6   # steps of ~1e-9 against tangential displacements of ~1e-3
    for _ in range(5):
        dx = rng.standard_normal(xh.shape) * 1e-3
        fd = (fr_.energy(f, xh + hh * dx) - fr_.energy(f, xh - hh * dx)) / (2 * hh)
        assert fd == pytest.approx(float(np.sum(G * dx)), rel=1e-6)
    for _ in range(5):
        dx = rng.standard_normal(xh.shape) * 1e-3
        Gp, Gm = np.zeros_like(xh), np.zeros_like(xh)
        fr_.add_to(f, xh + hh * dx, Gp, [], [], [])
        fr_.add_to(f, xh - hh * dx, Gm, [], [], [])
        fdg = ((Gp - Gm) / (2 * hh)).ravel()
        Hd = H @ dx.ravel()
        assert np.linalg.norm(fdg - Hd) <= 1e-5 * np.linalg.norm(Hd)


def test_tangent_basis_form_gives_the_same_terms():
    """IPC writes u = T^T v with an orthonormal tangent basis T (3x2); the
    projection form used here must give the same energy, gradient T grad_u and
    Hessian T H_u T^T, with H_u from the 2x2 formula in u."""
    sc, f = _sliding_scene(2)
    xh = sc["x_hat"]
    gv, Hv = fr_.terms(f, xh)
    e = f["e"]
    for i in range(len(f["ids"])):
        n = f["nrm"][i]
        a = np.array([1.0, 0, 0]) if abs(n[0]) < 0.9 else np.array([0, 1.0, 0])
        t1 = a - n * (a @ n)
        t1 /= np.linalg.norm(t1)
        T = np.stack([t1, np.cross(n, t1)], axis=1)
        v = f["w"][i] @ (xh[f["ids"][i]] - f["x0"][f["ids"][i]])
        u = T.T @ v
        y = np.linalg.norm(u)
        c = f["coef"][i]
        if y >= e:
            gu = c * u / y
            Hu = c * (np.eye(2) - np.outer(u, u) / y ** 2) / y
        else:
            gu = c * (2 / e - y / e ** 2) * u
            Hu = c * ((2 / e - y / e ** 2) * np.eye(2) - np.outer(u, u) / (y * e ** 2))
        assert np.allclose(T @ gu, gv[i], rtol=1e-10, atol=1e-14 * max(c, 1))
        assert np.allclose(T @ Hu @ T.T, Hv[i], rtol=1e-9, atol=1e-9 * np.abs(Hv[i]).max())


@pytest.mark.parametrize("L", [5e-3, 2e-3])
def test_kinetic_friction_closed_form(L):
    """A point of mass m whose inertial target lies L along the tangent plane
    (contact weights (1, 0, 0, 0)): minimizing m/2 |v - L t|^2 + coef f_0(|v_t|)
    gives, while sliding (L - coef/m > eps_v h), v = (L - coef / m) t: kinetic
    friction takes coef / m off the displacement."""
    m, coef, e = 2.0, 3e-3, 1e-4
    n = np.array([0.0, 0.0, 1.0])
    tdir = np.array([0.6, 0.8, 0.0])
    f = dict(ids=np.array([[0, 1, 2, 3]]), nrm=n[None], w=np.array([[1.0, 0.0, 0.0, 0.0]]),
             coef=np.array([coef]), x0=np.zeros((4, 3)), e=e)
    target = L * tdir
    v = np.zeros(3)
    xh = np.zeros((4, 3))
    for _ in range(100):
        xh[0] = v
        gv, Hv = fr_.terms(f, xh)
        g = m * (v - target) + gv[0]
        H = m * np.eye(3) + Hv[0]
        v = v - np.linalg.solve(H, g)
    assert np.allclose(v, (L - coef / m) * tdir, rtol=1e-10, atol=1e-15)


def test_static_friction_sticks_below_the_threshold():
    """The same point with coef / m > L: the displacement stays within the
    smoothing band |v_t| < eps_v h (static friction)."""
    m, coef, e = 2.0, 3e-2, 1e-4
    f = dict(ids=np.array([[0, 1, 2, 3]]), nrm=np.array([[0.0, 0.0, 1.0]]), w=np.array([[1.0, 0.0, 0.0, 0.0]]),
             coef=np.array([coef]), x0=np.zeros((4, 3)), e=e)
    target = np.array([5e-3, 0.0, 0.0])
    v = np.zeros(3)
    xh = np.zeros((4, 3))
    for _ in range(100):
        xh[0] = v
        gv, Hv = fr_.terms(f, xh)
        v = v - np.linalg.solve(m * np.eye(3) + Hv[0], m * (v - target) + gv[0])
    assert 0.0 < v[0] < e
    # stationarity: m (v - target) + coef f_1(y) = 0
    assert m * (v[0] - target[0]) + coef * float(fr_.f1(v[0], e)) == pytest.approx(0.0, abs=1e-12)


def test_assemble_with_friction_matches_total_energy_gradient():
    """The whole oracle G with the friction set is the gradient of its total energy."""
    sc, f = _sliding_scene(4)
    st = oracle.assemble(sc)
    free = ~sc["fixed"].astype(bool)
    rng = np.random.default_rng(5)
    hh = 1e-7
    prep = oracle.prepare(sc)
    for _ in range(3):
        dx = rng.standard_normal(sc["x_hat"].shape) * 1e-4 * free[:, None]
        fd = (oracle.total_energy(sc, prep, sc["x_hat"] + hh * dx)
              - oracle.total_energy(sc, prep, sc["x_hat"] - hh * dx)) / (2 * hh)
        assert fd == pytest.approx(float(np.sum(st.G * dx)), rel=1e-5)
    # a zero-coefficient set changes nothing
    sc0 = dict(sc, friction=dict(f, coef=np.zeros_like(f["coef"])))
    sc1 = {k: v for k, v in sc.items() if k != "friction"}
    assert np.array_equal(oracle.assemble(sc0).G, oracle.assemble(sc1).G)


def _slide_on_slope(mu_f, steps):
    """Time steps of the oracle (Algorithm 1 with friction, K_min = 6 as the
    paper uses with friction, mu_init at the first step) on scenes.slope;
    returns the upper cube's mean velocity along the slope after each step."""
    from oracle import timestep
    sc0 = scenes.slope()
    N, h, g = len(sc0["x"]), sc0["dt"], sc0["gravity"]
    up = np.arange(N) >= N // 2
    x, v = sc0["x"].copy(), np.zeros_like(sc0["x"])
    pt = ee = np.zeros((0, 4), dtype=np.int64)
    lam = gam = np.zeros(0)
    kappa, delta = sc0["kappa"], sc0["delta"]
    vs = []
    for step in range(steps):
        xt = x + h * v
        xt[up] += h * h * g
        sc = dict(sc0, x=x, x_hat=x.copy(), x_tilde=xt, pt=pt, ee=ee, lam=lam, gamma=gam, kappa=kappa, delta=delta)
        x, v, (pt, ee, lam, gam), info = timestep.time_step(sc, K_min=6, mu_f=mu_f, eps_v=1e-3,
                                                              mu_init_C=0.1 if step == 0 else None)
        kappa, delta = info["kappa"], info["delta"]
        vs.append(v[up, 0].mean())
    return np.array(vs), h


def test_block_on_slope_slides_at_the_analytic_acceleration():
    """Section 6's cubes on a slope (incline arctan 0.5): with mu_f = 0.3 below
    tan(theta) = 0.5 the block slides at g (sin - mu_f cos); its acceleration,
    once the contact force has settled at the weight (from the sixth step),
    agrees within 3 %."""
    vs, h = _slide_on_slope(0.3, 12)
    th = np.arctan(0.5)
    a = (vs[-1] - vs[5]) / (h * (len(vs) - 6))
    assert a == pytest.approx(9.8 * (np.sin(th) - 0.3 * np.cos(th)), rel=0.03)


def test_momentum_conservation_with_friction():
    """Section 6's momentum conservation in the oracle's time steps: two free
    cubes, the upper thrown onto the lower, friction on.  Every force is
    internal (constraint and friction weights sum to zero, energies are
    translation invariant), and the oracle's Newton steps solve exactly, so
    the total momentum stays at its initial value to rounding, while friction
    drags the lower cube sideways."""
    from oracle import timestep
    sc0 = dict(scenes.falling_cubes(jitter=1e-5))
    N, h = len(sc0["x"]), sc0["dt"]
    up = np.arange(N) >= N // 2
    sc0["fixed"] = np.zeros(N, dtype=np.uint8)
    m = oracle.prepare(sc0).mass
    x, v = sc0["x"].copy(), np.zeros_like(sc0["x"])
    v[up] = [0.2, 0.0, -0.5]
    P0 = (m[:, None] * v).sum(0)
    pt = ee = np.zeros((0, 4), dtype=np.int64)
    lam = gam = np.zeros(0)
    for _ in range(3):
        sc = dict(sc0, x=x, x_hat=x.copy(), x_tilde=x + h * v, pt=pt, ee=ee, lam=lam, gamma=gam)
        x, v, (pt, ee, lam, gam), _ = timestep.time_step(sc, K_min=6, mu_f=0.5, eps_v=1e-3)
    P = (m[:, None] * v).sum(0)
    assert np.abs(P - P0).max() <= 1e-12 * np.abs(P0).max()
    assert v[~up].mean(0)[0] > 0.005
