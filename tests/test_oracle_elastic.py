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


# ---------------------------------------------------------------- stable Neo-Hookean

def _rand_F(rng, n, scale=0.3):
    F = np.eye(3)[None] + scale * rng.standard_normal((n, 3, 3))
    F = F[np.linalg.det(F) > 0.2]
    return F


def test_snh_rest_and_uniform_scaling():
    mu, lam = np.array([3.0]), np.array([7.0])
    I = np.eye(3)[None]
    assert oracle.core.snh_energy(I, mu, lam)[0] == 0.0
    assert np.abs(oracle.core.snh_stress(I, mu, lam)).max() < 1e-15
    for s_ in (0.7, 1.0, 1.3):
        F = s_ * I
        ref = 1.5 * 3.0 * (s_ ** 2 - 1) - 3.0 * (s_ ** 3 - 1) + 0.5 * 7.0 * (s_ ** 3 - 1) ** 2
        assert oracle.core.snh_energy(F, mu, lam)[0] == pytest.approx(ref, rel=1e-13, abs=1e-14)


def test_snh_stress_and_hessian_are_derivatives():
    rng = np.random.default_rng(21)
    F = _rand_F(rng, 20)
    n = len(F)
    mu, lam = rng.uniform(1, 5, n), rng.uniform(1, 20, n)
    P = oracle.core.snh_stress(F, mu, lam)
    eps = 1e-6
    for k in range(9):
        E = np.zeros((n, 3, 3))
        E[:, k // 3, k % 3] = 1.0
        fd = (oracle.core.snh_energy(F + eps * E, mu, lam) - oracle.core.snh_energy(F - eps * E, mu, lam)) / (2 * eps)
        assert np.allclose(fd, P[:, k // 3, k % 3], rtol=1e-7, atol=1e-7)
        dP = oracle.core.snh_dP(F, E, mu, lam)
        fdP = (oracle.core.snh_stress(F + eps * E, mu, lam) - oracle.core.snh_stress(F - eps * E, mu, lam)) / (2 * eps)
        assert np.allclose(fdP, dP, rtol=1e-6, atol=1e-6)


def test_snh_rotation_invariance():
    rng = np.random.default_rng(22)
    F = _rand_F(rng, 10)
    n = len(F)
    mu, lam = np.full(n, 2.0), np.full(n, 9.0)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    R = Q * np.sign(np.linalg.det(Q))
    RF = R[None] @ F
    assert np.allclose(oracle.core.snh_energy(RF, mu, lam), oracle.core.snh_energy(F, mu, lam), rtol=1e-12)
    assert np.allclose(oracle.core.snh_stress(RF, mu, lam), R[None] @ oracle.core.snh_stress(F, mu, lam), atol=1e-12)


def test_snh_analytic_eigensystem_matches_the_numeric_hessian():
    """The closed forms the element kernel uses, derived for Psi = m(sigma) +
    g(J) with q = J g'(J), r = J^2 g''(J) (SNH: q = J (lam (J - 1) - mu),
    r = lam J^2): the 3x3 Hessian in the singular values has diagonal
    mu + r / s_i^2 and off-diagonal (r + q) / (s_i s_j); the pair modes are
    mu + q / (s_i s_j) and mu - q / (s_i s_j).  Their nine values equal the
    eigenvalues of the oracle's 9x9 d2Psi/dF2."""
    rng = np.random.default_rng(23)
    F = _rand_F(rng, 30, 0.4)
    n = len(F)
    mu, lam = rng.uniform(1, 5, n), rng.uniform(1, 20, n)
    H9 = oracle.core.nh_hessian9(F, mu, lam, np.ones(n))
    for e in range(n):
        s_ = np.linalg.svd(F[e], compute_uv=False)
        J = np.linalg.det(F[e])
        q = J * (lam[e] * (J - 1) - mu[e])
        r = lam[e] * J * J
        Hs = np.array([[mu[e] + r / s_[i] ** 2 if i == j else (r + q) / (s_[i] * s_[j]) for j in range(3)]
                       for i in range(3)])
        vals = list(np.linalg.eigvalsh(Hs))
        for i, j in ((0, 1), (0, 2), (1, 2)):
            vals += [mu[e] + q / (s_[i] * s_[j]), mu[e] - q / (s_[i] * s_[j])]
        num = np.linalg.eigvalsh(H9[e])
        assert np.allclose(np.sort(vals), num, rtol=1e-9, atol=1e-9 * np.abs(num).max())


def _rotations(rng, n):
    Q, _ = np.linalg.qr(rng.standard_normal((n, 3, 3)))
    return Q * np.sign(np.linalg.det(Q))[:, None, None]


def test_cor_closed_form_from_a_known_polar_pair():
    """F built as R S from a rotation R and an SPD S fixes the polar factors, so
    Psi = mu ||S - I||^2 + lam/2 tr(S - I)^2 and P = 2 mu R (S - I) + lam tr(S - I) R
    exactly (||F - R|| = ||R (S - I)|| = ||S - I||)."""
    rng = np.random.default_rng(31)
    n = 25
    R = _rotations(rng, n)
    B = rng.standard_normal((n, 3, 3)) * 0.25
    S = np.eye(3)[None] + 0.5 * (B + np.transpose(B, (0, 2, 1)))
    S = S[np.all(np.linalg.eigvalsh(S) > 0.2, axis=1)]
    R = R[:len(S)]
    n = len(S)
    F = R @ S
    mu, lam = rng.uniform(1, 5, n), rng.uniform(1, 20, n)
    D = S - np.eye(3)[None]
    tr = np.einsum("tii->t", D)
    psi = mu * np.einsum("tij,tij->t", D, D) + 0.5 * lam * tr ** 2
    P = 2.0 * mu[:, None, None] * (R @ D) + (lam * tr)[:, None, None] * R
    assert np.allclose(oracle.core.cor_energy(F, mu, lam), psi, rtol=1e-12, atol=1e-14)
    assert np.allclose(oracle.core.cor_stress(F, mu, lam), P, rtol=1e-12, atol=1e-13)
    I = np.eye(3)[None]
    assert oracle.core.cor_energy(I, mu[:1], lam[:1])[0] == 0.0
    assert np.abs(oracle.core.cor_stress(I, mu[:1], lam[:1])).max() < 1e-15


def test_cor_stress_and_hessian_are_derivatives():
    rng = np.random.default_rng(32)
    F = _rand_F(rng, 20)
    n = len(F)
    mu, lam = rng.uniform(1, 5, n), rng.uniform(1, 20, n)
    P = oracle.core.cor_stress(F, mu, lam)
    eps = 1e-6
    for k in range(9):
        E = np.zeros((n, 3, 3))
        E[:, k // 3, k % 3] = 1.0
        fd = (oracle.core.cor_energy(F + eps * E, mu, lam) - oracle.core.cor_energy(F - eps * E, mu, lam)) / (2 * eps)
        assert np.allclose(fd, P[:, k // 3, k % 3], rtol=1e-7, atol=1e-7)
        dP = oracle.core.cor_dP(F, E, mu, lam)
        fdP = (oracle.core.cor_stress(F + eps * E, mu, lam) - oracle.core.cor_stress(F - eps * E, mu, lam)) / (2 * eps)
        assert np.allclose(fdP, dP, rtol=1e-6, atol=1e-6)


def test_cor_rotation_invariance():
    rng = np.random.default_rng(33)
    F = _rand_F(rng, 10)
    n = len(F)
    mu, lam = np.full(n, 2.0), np.full(n, 9.0)
    R = _rotations(rng, 1)[0]
    RF = R[None] @ F
    assert np.allclose(oracle.core.cor_energy(RF, mu, lam), oracle.core.cor_energy(F, mu, lam), rtol=1e-12)
    assert np.allclose(oracle.core.cor_stress(RF, mu, lam), R[None] @ oracle.core.cor_stress(F, mu, lam), atol=1e-12)


def test_cor_analytic_eigensystem_matches_the_numeric_hessian():
    """The closed forms the element kernel uses for Psi = mu sum (s_i - 1)^2 +
    lam/2 (sum s_i - 3)^2: the 3x3 Hessian in the singular values is
    2 mu I + lam 1 1^T; with Psi_i = 2 mu (s_i - 1) + lam (sum s - 3) the pair
    modes are (Psi_i + Psi_j) / (s_i + s_j) and (Psi_i - Psi_j) / (s_i - s_j) = 2 mu.
    Their nine values equal the eigenvalues of the oracle's 9x9 d2Psi/dF2."""
    rng = np.random.default_rng(34)
    F = _rand_F(rng, 30, 0.4)
    n = len(F)
    mu, lam = rng.uniform(1, 5, n), rng.uniform(1, 20, n)
    H9 = oracle.core.nh_hessian9(F, mu, lam, np.full(n, 2))
    for e in range(n):
        s_ = np.linalg.svd(F[e], compute_uv=False)
        t = s_.sum() - 3.0
        dpsi = 2.0 * mu[e] * (s_ - 1.0) + lam[e] * t
        vals = list(np.linalg.eigvalsh(2.0 * mu[e] * np.eye(3) + lam[e] * np.ones((3, 3))))
        for i, j in ((0, 1), (0, 2), (1, 2)):
            vals += [(dpsi[i] + dpsi[j]) / (s_[i] + s_[j]), 2.0 * mu[e]]
        num = np.linalg.eigvalsh(H9[e])
        assert np.allclose(np.sort(vals), num, rtol=1e-9, atol=1e-9 * np.abs(num).max())


def test_material_dispatch_per_tet():
    """psi_* pick each tet's own material (codes 0, 1, 2) in one call."""
    rng = np.random.default_rng(35)
    F = _rand_F(rng, 12)
    n = len(F)
    mu, lam = rng.uniform(1, 5, n), rng.uniform(1, 20, n)
    mat = np.arange(n) % 3
    E = oracle.core.psi_energy(F, mu, lam, mat)
    P = oracle.core.psi_stress(F, mu, lam, mat)
    for code, fe, fs in ((0, oracle.core.nh_energy, oracle.core.nh_stress),
                         (1, oracle.core.snh_energy, oracle.core.snh_stress),
                         (2, oracle.core.cor_energy, oracle.core.cor_stress)):
        k = mat == code
        assert np.array_equal(E[k], fe(F[k], mu[k], lam[k]))
        assert np.array_equal(P[k], fs(F[k], mu[k], lam[k]))
