"""Pins of the oracle's geometry, mass and Neo-Hookean elasticity against
closed forms, finite differences and an independently derived eigensystem."""
import numpy as np
import pytest

import oracle
from scenes import kuhn_cube

RNG = np.random.default_rng(7)


def rand_rot(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    return q


def rand_F(rng, n, spread=0.3):
    F = np.eye(3) + spread * rng.normal(size=(n, 3, 3))
    F[np.linalg.det(F) < 0, :, 0] *= -1
    return F


def mats(n, E=1e5, nu=0.4):
    mu, lam = oracle.lame(np.full(n, E), np.full(n, nu))
    return mu, lam


# ---------------------------------------------------------------- geometry ---

def test_kuhn_volumes_and_mass():
    a, n, rho = 0.25, 4, 1000.0
    X, T = kuhn_cube(n, a)
    Dminv, vol, A = oracle.rest_geometry(X, T.astype(np.int64))
    assert np.allclose(vol, a ** 3 / 6, rtol=1e-13)          # each Kuhn tet is a^3/6
    assert np.isclose(vol.sum(), (n * a) ** 3, rtol=1e-13)    # they tile the cube
    m = oracle.lumped_mass(len(X), T, vol, np.full(len(T), rho))
    assert np.isclose(m.sum(), rho * (n * a) ** 3, rtol=1e-13)
    # the A rows map vertex displacements to dF: a rigid translation gives dF = 0
    assert np.allclose(A.sum(axis=1), 0.0, atol=1e-12)
    # and the rest edges map to the identity: sum_a X_a (outer) A_a = I
    F = np.einsum("tai,taj->tij", X[T], A)
    assert np.allclose(F, np.eye(3), atol=1e-12)


def test_lame():
    mu, lam = oracle.lame(np.array([1e5]), np.array([0.4]))
    assert np.isclose(mu[0], 1e5 / 2.8) and np.isclose(lam[0], 1e5 * 0.4 / (1.4 * 0.2))


# ------------------------------------------------------------- Neo-Hookean ---

def test_rest_state_zero_energy_and_stress():
    F = np.repeat(np.eye(3)[None], 4, axis=0)
    mu, lam = mats(4)
    assert np.allclose(oracle.nh_energy(F, mu, lam), 0.0, atol=1e-12)
    assert np.allclose(oracle.nh_stress(F, mu, lam), 0.0, atol=1e-9)


def test_uniform_scaling_closed_form():
    s = np.array([0.6, 0.9, 1.0, 1.3])
    F = s[:, None, None] * np.eye(3)[None]
    mu, lam = mats(4)
    want = 1.5 * mu * (s ** 2 - 1) - 3 * mu * np.log(s) + 4.5 * lam * np.log(s) ** 2
    assert np.allclose(oracle.nh_energy(F, mu, lam), want, rtol=1e-12)
    # P = (mu (s - 1/s) + 3 lam ln s / s) I
    Pw = (mu * (s - 1 / s) + 3 * lam * np.log(s) / s)[:, None, None] * np.eye(3)
    assert np.allclose(oracle.nh_stress(F, mu, lam), Pw, rtol=1e-12, atol=1e-9)


def test_rotation_invariance_and_covariance():
    F = rand_F(RNG, 16)
    mu, lam = mats(16)
    R = np.stack([rand_rot(RNG) for _ in range(16)])
    assert np.allclose(oracle.nh_energy(R @ F, mu, lam), oracle.nh_energy(F, mu, lam), rtol=1e-11)
    assert np.allclose(oracle.nh_stress(R @ F, mu, lam), R @ oracle.nh_stress(F, mu, lam),
                       rtol=1e-9, atol=1e-6)


def test_stress_is_energy_gradient_fd():
    F = rand_F(RNG, 8)
    mu, lam = mats(8)
    P = oracle.nh_stress(F, mu, lam)
    eps = 1e-6
    for i in range(3):
        for j in range(3):
            dF = np.zeros_like(F)
            dF[:, i, j] = eps
            fd = (oracle.nh_energy(F + dF, mu, lam) - oracle.nh_energy(F - dF, mu, lam)) / (2 * eps)
            assert np.allclose(fd, P[:, i, j], rtol=1e-7, atol=1e-3)


def test_hessian9_is_stress_derivative_fd_and_symmetric():
    F = rand_F(RNG, 8)
    mu, lam = mats(8)
    H = oracle.nh_hessian9(F, mu, lam)
    Hraw = np.stack([oracle.nh_dP(F, np.eye(9)[k].reshape(1, 3, 3).repeat(8, 0), mu, lam).reshape(8, 9)
                     for k in range(9)], axis=2)
    assert np.allclose(Hraw, np.transpose(Hraw, (0, 2, 1)), rtol=1e-10, atol=1e-5)
    eps = 1e-6
    for k in range(9):
        dF = np.zeros((8, 9))
        dF[:, k] = eps
        dF = dF.reshape(8, 3, 3)
        fd = (oracle.nh_stress(F + dF, mu, lam) - oracle.nh_stress(F - dF, mu, lam)).reshape(8, 9) / (2 * eps)
        assert np.allclose(fd, H[:, :, k], rtol=1e-6, atol=1e-2 * mu[0] * 1e-4)


def _analytic_projected(F, mu, lam):
    """Independent derivation: the 9 eigenpairs of d2Psi/dF2 in the SVD frame
    (3 scaling modes from the 3x3 Hessian in singular values, 3 twist and 3 flip
    modes), clamped at zero and summed as omega+ vec(Q) vec(Q)^T."""
    out = np.empty((len(F), 9, 9))
    for t in range(len(F)):
        U, S, Vt = np.linalg.svd(F[t])
        if np.linalg.det(U) < 0:
            U[:, 2] *= -1
            S[2] *= -1
        if np.linalg.det(Vt) < 0:
            Vt[2, :] *= -1
            S[2] *= -1
        m, l = mu[t], lam[t]
        lnJ = np.log(np.prod(S))
        Ahat = np.empty((3, 3))
        for i in range(3):
            for j in range(3):
                Ahat[i, j] = m + (m + l - l * lnJ) / S[i] ** 2 if i == j else l / (S[i] * S[j])
        w, e = np.linalg.eigh(Ahat)
        H = np.zeros((9, 9))
        for k in range(3):
            Q = U @ np.diag(e[:, k]) @ Vt
            H += max(w[k], 0) * np.outer(Q.ravel(), Q.ravel())
        for (i, j) in ((0, 1), (0, 2), (1, 2)):
            D = np.zeros((3, 3))
            D[i, j], D[j, i] = 1 / np.sqrt(2), -1 / np.sqrt(2)
            wt = m + (l * lnJ - m) / (S[i] * S[j])
            Q = U @ D @ Vt
            H += max(wt, 0) * np.outer(Q.ravel(), Q.ravel())
            D[j, i] = 1 / np.sqrt(2)
            wf = m + (m - l * lnJ) / (S[i] * S[j])
            Q = U @ D @ Vt
            H += max(wf, 0) * np.outer(Q.ravel(), Q.ravel())
        out[t] = H
    return out


@pytest.mark.parametrize("kind", ["random", "compressed", "repeated", "stretched"])
def test_numeric_clamp_matches_analytic_eigensystem(kind):
    n = 12
    if kind == "random":
        F = rand_F(RNG, n)
    elif kind == "compressed":
        F = np.stack([rand_rot(RNG) @ np.diag([1.0, 1.0, 0.6]) @ rand_rot(RNG) for _ in range(n)])
    elif kind == "repeated":
        F = np.stack([rand_rot(RNG) @ np.diag([0.8, 0.8, 0.8 + 1e-9]) @ rand_rot(RNG) for _ in range(n)])
    else:
        F = np.stack([rand_rot(RNG) @ np.diag([3.0, 2.5, 2.0]) @ rand_rot(RNG) for _ in range(n)])
    mu, lam = mats(n)
    raw = oracle.nh_hessian9(F, mu, lam)
    if kind == "compressed":   # the clamp must actually act in this case
        assert np.linalg.eigvalsh(raw).min() < 0
    num = oracle.psd_project(raw)
    ana = _analytic_projected(F, mu, lam)
    scale = np.abs(ana).max()
    assert np.abs(num - ana).max() <= 1e-9 * scale
    ev = np.linalg.eigvalsh(num)
    assert ev.min() >= -1e-12 * np.abs(ev).max()


def test_projection_inactive_at_rest():
    F = np.repeat(np.eye(3)[None], 3, axis=0)
    mu, lam = mats(3)
    H = oracle.nh_hessian9(F, mu, lam)
    assert np.allclose(oracle.psd_project(H), H, atol=1e-9 * np.abs(H).max())


def test_element_hessian_nullspace_covariance_and_block_identity():
    X, T = kuhn_cube(1, 0.5)
    T = T.astype(np.int64)
    Dminv, vol, A = oracle.rest_geometry(X, T)
    mu, lam = mats(len(T))
    xh = X + 0.05 * RNG.normal(size=X.shape)
    xh[:, 2] *= 0.7                                   # compress so the clamp is active
    g, He = oracle.elastic_terms(xh, T, Dminv, vol, A, mu, lam, 0.01)
    # translations are in the null space of every element Hessian and the gradient sums to 0
    for t in np.eye(3):
        assert np.abs(He @ np.tile(t, 4)).max() <= 1e-10 * np.abs(He).max()
    assert np.abs(g.sum(axis=1)).max() <= 1e-10 * np.abs(g).max()
    # rotating the deformed state rotates the gradient and the Hessian
    R = rand_rot(RNG)
    g2, He2 = oracle.elastic_terms(xh @ R.T, T, Dminv, vol, A, mu, lam, 0.01)
    R4 = np.kron(np.eye(4), R)
    assert np.allclose(g2, g @ R.T, rtol=1e-9, atol=1e-9 * np.abs(g).max())
    assert np.allclose(He2, R4 @ He @ R4.T, atol=1e-9 * np.abs(He).max())
    # gradient matches finite differences of h^2 V Psi
    F = oracle.deformation_gradient(xh, T, Dminv)
    eps = 1e-7
    Xe = xh[T].copy()

    def psi(Xe_):
        Ds = np.stack([Xe_[:, 1] - Xe_[:, 0], Xe_[:, 2] - Xe_[:, 0], Xe_[:, 3] - Xe_[:, 0]], axis=2)
        return 0.01 ** 2 * vol * oracle.nh_energy(Ds @ Dminv, mu, lam)

    for a in range(4):
        for i in range(3):
            # per-element FD: perturb vertex a of each element independently
            Xp, Xm = Xe.copy(), Xe.copy()
            Xp[:, a, i] += eps
            Xm[:, a, i] -= eps
            fd = (psi(Xp) - psi(Xm)) / (2 * eps)
            assert np.allclose(fd, g[:, a, i], rtol=1e-5, atol=1e-6 * np.abs(g).max())
    # the paper's vertex-block identity (Section 5.1) equals the dense B^T H9+ B
    for t in range(len(T)):
        U, S, Vt = np.linalg.svd(F[t])
        if np.linalg.det(U) < 0:
            U[:, 2] *= -1
            S[2] *= -1
        if np.linalg.det(Vt) < 0:
            Vt[2, :] *= -1
            S[2] *= -1
        V = Vt.T
        m, l = mu[t], lam[t]
        lnJ = np.log(np.prod(S))
        Ahat = np.array([[m + (m + l - l * lnJ) / S[i] ** 2 if i == j else l / (S[i] * S[j])
                          for j in range(3)] for i in range(3)])
        w, e = np.linalg.eigh(Ahat)
        modes = [(max(w[k], 0), np.diag(e[:, k])) for k in range(3)]
        for (i, j) in ((0, 1), (0, 2), (1, 2)):
            D = np.zeros((3, 3))
            D[i, j], D[j, i] = 1 / np.sqrt(2), -1 / np.sqrt(2)
            modes.append((max(m + (l * lnJ - m) / (S[i] * S[j]), 0), D.copy()))
            D[j, i] = 1 / np.sqrt(2)
            modes.append((max(m + (m - l * lnJ) / (S[i] * S[j]), 0), D.copy()))
        for a in range(4):
            for b in range(4):
                va = (A[t, a] @ V)[None, :]
                vb = (A[t, b] @ V)[None, :]
                inner = sum(wk * Dk @ va.T @ vb @ Dk.T for wk, Dk in modes)
                blk = 0.01 ** 2 * vol[t] * U @ inner @ U.T
                ref = He[t, 3 * a:3 * a + 3, 3 * b:3 * b + 3]
                assert np.allclose(blk, ref, atol=1e-9 * np.abs(He[t]).max())


def test_inverted_element_raises():
    F = np.diag([1.0, 1.0, -0.5])[None]
    mu, lam = mats(1)
    with pytest.raises(ValueError):
        oracle.nh_stress(F, mu, lam)
