"""Pins of the oracle's SolveSubproblem pieces (Algorithm 2 after the Newton
step): the multiplier/decay update, the halving line search and the Newton
loop."""
import numpy as np
import pytest

import oracle
from oracle import subproblem as osp
import scenes

RNG = np.random.default_rng(11)


@pytest.fixture(scope="module")
def shifted():
    return scenes.tiny(lateral=(0.37, 0.21))


def test_dual_update_is_the_projected_multiplier_update(shifted):
    """Algorithm 2's branch on s_i equals the textbook projected update
    lambda' = max(0, lambda - mu c) of the augmented Lagrangian method for
    c_i >= 0 constraints, with gamma' = 1 exactly where that update is active."""
    sc = dict(shifted)
    mu = sc["kappa"]
    for scale in (1e-4, 1e-3, 5e-3):
        xh = sc["x_hat"] + scale * RNG.normal(size=sc["x_hat"].shape) * (1 - sc["fixed"])[:, None]
        gam = RNG.uniform(0.2, 1.0, size=len(sc["lam"]))
        sc["gamma"] = gam
        # half of the multipliers zero, so both branches of the update occur
        sc["lam"] = shifted["lam"] * (RNG.random(len(gam)) < 0.5)
        lam2, gam2, active = osp.dual_update(sc, xh, Gamma=0.9)
        c = osp.constraint_values_at(sc, xh)
        textbook = np.maximum(0.0, sc["lam"] - mu * c)
        assert np.allclose(lam2, textbook, rtol=1e-12, atol=1e-9)
        assert np.all(lam2 >= 0.0)
        assert np.array_equal(active, sc["lam"] - mu * c >= 0.0)
        assert np.all(gam2[active] == 1.0) and np.allclose(gam2[~active], 0.9 * gam[~active])
        assert 0 < active.sum() < len(active)


def test_line_search_takes_the_first_halving_that_decreases_energy(shifted):
    st = oracle.assemble(shifted)
    prep = oracle.prepare(shifted)
    xh = shifted["x_hat"]
    p = oracle.solve_direct(st.H, st.G)
    L0 = osp.energy(shifted, prep, xh)
    r, L1 = osp.line_search(shifted, prep, xh, p, L0)
    assert 0.0 < r <= 1.0 and L1 < L0
    assert L1 == osp.energy(shifted, prep, xh + r * p)
    # a step 64 times too long must be cut back, to the first power of two that decreases L
    r2, L2 = osp.line_search(shifted, prep, xh, 64.0 * p, L0)
    assert r2 < 1.0 and L2 < L0
    assert osp.energy(shifted, prep, xh + 2.0 * r2 * 64.0 * p) >= L0
    # an ascent direction never decreases L: the search gives up with r = 0
    g = st.G / np.linalg.norm(st.G)
    r3, L3 = osp.line_search(shifted, prep, xh, 1e-6 * g, L0)
    assert (r3, L3) == (0.0, L0)


def test_inverted_trial_counts_as_infinite_energy(shifted):
    prep = oracle.prepare(shifted)
    xh = shifted["x_hat"].copy()
    t = shifted["tets"][0]
    bad = xh.copy()
    bad[t[0]] = xh[t[1]] + 2.0 * (xh[t[1]] - xh[t[0]])
    assert osp.energy(shifted, prep, bad) == np.inf


def test_newton_loop_decreases_energy_and_ends_on_a_full_step(shifted):
    xh, lam, gam, hist = osp.solve_subproblem(shifted, max_newton=20)
    assert len(hist) >= 1
    for L0, r, L1 in hist:
        assert L1 < L0 and 0.0 < r <= 1.0
    assert hist[-1][1] == 1.0
    # the gradient after the loop is much smaller than at x_hat^0 (the energy is only C1
    # where a constraint switches between its quadratic and constant branches)
    sc = dict(shifted)
    sc["x_hat"] = xh
    g1 = oracle.assemble(sc).G
    g0 = oracle.assemble(shifted).G
    assert np.linalg.norm(g1) < 0.25 * np.linalg.norm(g0)
    assert np.all(xh[shifted["fixed"].astype(bool)] == shifted["x_hat"][shifted["fixed"].astype(bool)])


def test_repeated_subproblems_drive_constraints_to_feasibility():
    """The augmented-Lagrangian outer iteration (subproblem, then multiplier
    update) makes the linearized constraints c_i >= 0 hold to a shrinking
    violation while the multipliers settle (Section 4.2)."""
    sc = scenes.tiny(lateral=(0.37, 0.21))
    # push the upper cube into the lower one so the constraints must act
    sc = dict(sc)
    push = np.zeros_like(sc["x_hat"])
    upper = sc["rest"][:, 2] > 1.0
    push[upper, 2] = -0.004
    sc["x_hat"] = sc["x_hat"] + push
    sc["x_tilde"] = sc["x_tilde"] + push
    sc["lam"] = np.zeros_like(sc["lam"])
    viol = []
    for _ in range(6):
        xh, lam, gam, _ = osp.solve_subproblem(sc, max_newton=20)
        c = osp.constraint_values_at(sc, xh)
        viol.append(float(np.maximum(0.0, -c).max()))
        sc["x_hat"], sc["lam"], sc["gamma"] = xh, lam, gam
    assert viol[0] > 0.0
    assert viol[-1] < 0.1 * viol[0]


def _kuhn_linear_elastic_diagonal(sc):
    """The Hessian diagonal at rest written out from the rest shape alone: at
    F = I the Neo-Hookean second variation is that of linear elasticity,
    mu |dF|^2 + mu dF:dF^T + lambda tr(dF)^2, and moving vertex a of a tet
    along axis i gives dF = e_i a_a^T (a_a the rows of D_m^-1, a_0 = -sum), so
    the entry is m_v + h^2 sum_e V_e (mu |a_a|^2 + (mu + lambda) a_{a,i}^2)."""
    rest, tets = sc["rest"], sc["tets"]
    N = len(rest)
    diag = np.zeros(3 * N)
    for k, t in enumerate(tets):
        X = rest[t]
        Dm = np.column_stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]])
        V = abs(np.linalg.det(Dm)) / 6.0
        Ai = np.linalg.inv(Dm)
        a = [-(Ai[0] + Ai[1] + Ai[2]), Ai[0], Ai[1], Ai[2]]
        E, nu, rho = sc["E"][k], sc["nu"][k], sc["rho"][k]
        mu = E / (2 * (1 + nu))
        lam = E * nu / ((1 + nu) * (1 - 2 * nu))
        for v in range(4):
            for i in range(3):
                diag[3 * t[v] + i] += rho * V / 4 + sc["dt"] ** 2 * V * (mu * a[v] @ a[v] + (mu + lam) * a[v][i] ** 2)
    return diag


def test_hessian_diagonal_at_rest_is_the_linear_elastic_closed_form():
    sc = scenes.tiny()
    assert np.array_equal(sc["x"], sc["rest"])
    st = oracle.prepare(sc)
    d = osp.hessian_diagonal(sc, st, sc["x"])
    ref = _kuhn_linear_elastic_diagonal(sc)
    assert np.allclose(d, ref, rtol=1e-12, atol=0.0)
    mu0 = osp.mu_init(sc)
    assert mu0 == pytest.approx(0.1 * ref.max(), rel=1e-12)
    print(f"tiny: mu_init = {mu0:.4f} (the configuration's kappa is {sc['kappa']:.0e})")


def test_hessian_diagonal_is_the_second_derivative_of_the_energy():
    """At a deformed state where no element's projection is active the
    diagonal equals the central second difference of E = 1/2 |x - x_tilde|_M^2
    + h^2 sum V Psi along each coordinate (checked at the largest entry and at
    random ones).  Near rest any compression (J < 1) makes the twist modes
    negative (omega ~ lambda ln J), so the state is a 5 % dilation with noise."""
    sc = dict(scenes.tiny(lateral=(0.37, 0.21)))
    sc["pt"] = np.zeros((0, 4), np.int32)
    sc["ee"] = np.zeros((0, 4), np.int32)
    sc["lam"] = np.zeros(0)
    sc["gamma"] = np.zeros(0)
    st = oracle.prepare(sc)
    xs = 1.05 * sc["rest"] + 1e-3 * RNG.standard_normal(sc["rest"].shape)
    F = oracle.core.deformation_gradient(xs, st.tets, st.Dminv)
    ev = np.linalg.eigvalsh(oracle.core.nh_hessian9(F, st.mu_l, st.lam_l))
    assert ev.min() > 0.0, "the projection must be inactive for this pin"
    d = osp.hessian_diagonal(sc, st, xs)
    eps = 1e-4
    for j in [int(np.argmax(d))] + list(RNG.choice(3 * len(xs), 8, replace=False)):
        v, i = divmod(j, 3)
        f = []
        for s in (-1, 0, 1):
            x2 = xs.copy()
            x2[v, i] += s * eps
            f.append(oracle.total_energy(sc, st, x2))
        fd = (f[0] - 2 * f[1] + f[2]) / eps ** 2
        assert fd == pytest.approx(d[j], rel=1e-5), (j, fd, d[j])


def test_mu_init_is_taken_at_x_not_x_hat(shifted):
    sc = dict(shifted)
    m0 = osp.mu_init(sc)
    sc["x_hat"] = sc["x_hat"] + 0.01
    assert osp.mu_init(sc) == m0
    sc["x"] = sc["x"] * np.array([1.0, 1.0, 0.9])
    assert osp.mu_init(sc) != m0
