"""Pins of the oracle's point-triangle and edge-edge distances: closed forms,
brute-force minimization, finite differences and translation invariance."""
import numpy as np
import pytest

import oracle

RNG = np.random.default_rng(11)


def one(f, *pts):
    d, n, w = f(*[np.asarray(p, dtype=float)[None] for p in pts])
    return d[0], n[0], w[0]


def test_pt_closed_forms():
    t0, t1, t2 = (0, 0, 0), (1, 0, 0), (0, 1, 0)
    # above the interior: distance is the height, closest point (0.2, 0.3, 0)
    d, n, w = one(oracle.pt_closest, (0.2, 0.3, 0.7), t0, t1, t2)
    assert np.isclose(d, 0.7) and np.allclose(n, (0, 0, 1)) and np.allclose(w, (1, -0.5, -0.2, -0.3))
    # below the interior: normal flips
    d, n, w = one(oracle.pt_closest, (0.2, 0.3, -0.7), t0, t1, t2)
    assert np.isclose(d, 0.7) and np.allclose(n, (0, 0, -1))
    # off the hypotenuse edge: point-segment distance
    d, n, w = one(oracle.pt_closest, (1.0, 1.0, 0.5), t0, t1, t2)
    assert np.isclose(d, np.sqrt(0.5 + 0.25)) and np.allclose(w, (1, 0, -0.5, -0.5))
    # off a vertex region: point-point distance
    d, n, w = one(oracle.pt_closest, (-1.0, -2.0, 2.0), t0, t1, t2)
    assert np.isclose(d, 3.0) and np.allclose(w, (1, -1, 0, 0)) and np.allclose(n, np.array([-1, -2, 2]) / 3)


def test_ee_closed_forms():
    # perpendicular skew segments crossing at their midpoints, offset 0.4 in z
    d, n, w = one(oracle.ee_closest, (-1, 0, 0.4), (1, 0, 0.4), (0, -1, 0), (0, 1, 0))
    assert np.isclose(d, 0.4) and np.allclose(n, (0, 0, 1)) and np.allclose(w, (0.5, 0.5, -0.5, -0.5))
    # closest at an endpoint of one segment and interior of the other
    d, n, w = one(oracle.ee_closest, (2, 0, 0.3), (3, 0, 0.3), (0, -1, 0), (0, 1, 0))
    assert np.isclose(d, np.hypot(2, 0.3)) and np.allclose(w, (1, 0, -0.5, -0.5))
    # endpoint to endpoint
    d, n, w = one(oracle.ee_closest, (2, 2, 1), (3, 3, 1), (0, 0, 0), (-1, 0.5, 0))
    assert np.isclose(d, 3.0) and np.allclose(w, (1, 0, -1, 0))


def _brute_pt(p, t0, t1, t2, m=401):
    u = np.linspace(0, 1, m)
    U, V = np.meshgrid(u, u)
    ok = U + V <= 1
    U, V = U[ok], V[ok]
    Q = t0 + U[:, None] * (t1 - t0) + V[:, None] * (t2 - t0)
    k = np.argmin(np.linalg.norm(Q - p, axis=1))
    u0, v0, h = U[k], V[k], 2.0 / (m - 1)
    for _ in range(3):   # refine with successively finer local grids
        uu = np.clip(np.linspace(u0 - h, u0 + h, 101), 0, 1)
        vv = np.clip(np.linspace(v0 - h, v0 + h, 101), 0, 1)
        U, V = np.meshgrid(uu, vv)
        U, V = U.ravel(), V.ravel()
        ok = U + V <= 1
        U, V = U[ok], V[ok]
        Q = t0 + U[:, None] * (t1 - t0) + V[:, None] * (t2 - t0)
        D = np.linalg.norm(Q - p, axis=1)
        k = np.argmin(D)
        u0, v0, h = U[k], V[k], h / 25
    return D.min()


def _brute_ee(a0, a1, b0, b1, m=401):
    s = np.linspace(0, 1, m)
    S, T = np.meshgrid(s, s)
    P = a0 + S.ravel()[:, None] * (a1 - a0)
    Q = b0 + T.ravel()[:, None] * (b1 - b0)
    D = np.linalg.norm(P - Q, axis=1)
    k = np.argmin(D)
    s0, t0, h = S.ravel()[k], T.ravel()[k], 2.0 / (m - 1)
    for _ in range(3):   # refine with successively finer local grids
        ss = np.clip(np.linspace(s0 - h, s0 + h, 101), 0, 1)
        tt = np.clip(np.linspace(t0 - h, t0 + h, 101), 0, 1)
        S, T = np.meshgrid(ss, tt)
        S, T = S.ravel(), T.ravel()
        P = a0 + S[:, None] * (a1 - a0)
        Q = b0 + T[:, None] * (b1 - b0)
        D = np.linalg.norm(P - Q, axis=1)
        k = np.argmin(D)
        s0, t0, h = S[k], T[k], h / 25
    return D.min()


def test_brute_force_random():
    for _ in range(40):
        X = RNG.normal(size=(4, 3))
        d, n, w = one(oracle.pt_closest, *X)
        bp = _brute_pt(*X)
        assert bp - 1e-11 <= d <= bp + 1e-12
        d, n, w = one(oracle.ee_closest, *X)
        be = _brute_ee(*X)
        assert be - 1e-11 <= d <= be + 1e-12


@pytest.mark.parametrize("fn", [oracle.pt_closest, oracle.ee_closest])
def test_gradient_fd_and_translation_invariance(fn):
    X = RNG.normal(size=(64, 4, 3))
    d, n, w = fn(X[:, 0], X[:, 1], X[:, 2], X[:, 3])
    assert np.allclose(w.sum(axis=1), 0.0, atol=1e-14)           # sum_a w_a = 0
    assert np.allclose(np.linalg.norm(n, axis=1), 1.0)
    grad = w[:, :, None] * n[:, None, :]
    eps = 1e-6
    for a in range(4):
        for i in range(3):
            Xp, Xm = X.copy(), X.copy()
            Xp[:, a, i] += eps
            Xm[:, a, i] -= eps
            dp = fn(Xp[:, 0], Xp[:, 1], Xp[:, 2], Xp[:, 3])[0]
            dm = fn(Xm[:, 0], Xm[:, 1], Xm[:, 2], Xm[:, 3])[0]
            assert np.allclose((dp - dm) / (2 * eps), grad[:, a, i], atol=1e-7)
    # the distance is the distance between the reported closest points
    if fn is oracle.pt_closest:
        q = -(w[:, 1:2] * X[:, 1] + w[:, 2:3] * X[:, 2] + w[:, 3:4] * X[:, 3])
        assert np.allclose(np.linalg.norm(X[:, 0] - q, axis=1), d)
    else:
        P = w[:, 0:1] * X[:, 0] + w[:, 1:2] * X[:, 1]
        Q = -(w[:, 2:3] * X[:, 2] + w[:, 3:4] * X[:, 3])
        assert np.allclose(np.linalg.norm(P - Q, axis=1), d)
