"""The rest of SolveSubproblem (Algorithm 2) on the GPU against the FP64
oracle: the FP64 total energy, the Newton loop with its halving line search,
and the multiplier/decay update.

Bars: L within 1e-9 relative (both sides FP64); the subproblem's displacement
x_hat - x_hat^0 within 1e-4 of the oracle's in the energy norm of H at x_hat^0
(the GPU's Newton steps are PCG solves to 1e-7, the oracle's direct); the update
against the oracle's at the same x_hat as the shared checks state it (gamma
exact in its branch, lambda within 1e-9 relative plus kappa * 1e-11)."""
import numpy as np
import pytest

import oracle
from oracle import subproblem as osp
import scenes
from subproblem_checks import check_subproblem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bf():
    from paper_2512_12151_amd import bfal
    return bfal


@pytest.fixture(scope="module")
def ctx(bf):
    return bf.Context(0)


def pushed():
    """The shifted tiny stack with the upper cube pushed 4 mm into the lower one."""
    sc = dict(scenes.tiny(lateral=(0.37, 0.21)))
    push = np.zeros_like(sc["x_hat"])
    push[sc["rest"][:, 2] > 1.0, 2] = -0.004
    sc["x_hat"] = sc["x_hat"] + push
    sc["x_tilde"] = sc["x_tilde"] + push
    sc["lam"] = np.zeros_like(sc["lam"])
    return sc


def stretched():
    """The shifted tiny stack with h = 1 s and the lower cube stretched 1.8x in z
    (the upper one carried along): the first full Newton step overshoots and
    the line search halves it once."""
    sc = dict(scenes.tiny(lateral=(0.37, 0.21)))
    sc["dt"] = 1.0
    xh = sc["x"].copy()
    lower = sc["rest"][:, 2] <= 1.0
    xh[lower, 2] = sc["rest"][lower, 2] * 1.8
    xh[~lower, 2] = sc["rest"][~lower, 2] + 0.8
    sc["x_hat"] = np.where(sc["fixed"][:, None] == 1, sc["x"], xh)
    return sc


CASES = {"tiny_shifted": lambda: scenes.tiny(lateral=(0.37, 0.21)), "pushed": pushed, "stretched": stretched,
         "two_8cubes": lambda: scenes.tiny(n=8, n_pt=300, n_ee=200, lateral=(0.3, 0.6))}


@pytest.mark.parametrize("name", list(CASES) + ["medium"])
def test_energy_matches_oracle(ctx, bf, name):
    sc = CASES[name]() if name in CASES else scenes.medium()
    print(f"case {name}", flush=True)
    pb = bf.Problem.from_scene(ctx, sc)
    pb.newton_step(tol=1e-5)
    L, inv = pb.energy()
    Lref = oracle.total_energy(sc, oracle.prepare(sc), sc["x_hat"])
    print(f"{name}: L = {L:.15e}, oracle {Lref:.15e}", flush=True)
    assert not inv
    assert abs(L - Lref) <= 1e-9 * abs(Lref)


def test_inverted_state_has_infinite_energy(ctx, bf):
    sc = scenes.tiny(lateral=(0.37, 0.21))
    pb = bf.Problem.from_scene(ctx, sc)
    pb.newton_step(tol=1e-5)
    xh = sc["x_hat"].copy()
    t = sc["tets"][0]
    xh[t[0]] = xh[t[1]] + 2.0 * (xh[t[1]] - xh[t[0]])
    pb.set_state(sc["x"], xh, sc["x_tilde"], sc["dt"])
    L, inv = pb.energy()
    assert inv and L == np.inf


@pytest.mark.parametrize("name", list(CASES))
def test_subproblem_matches_oracle(ctx, bf, name):
    sc = CASES[name]()
    print(f"case {name}", flush=True)
    xr, lam_r, gam_r, hist = osp.solve_subproblem(sc, max_newton=20)
    pb = bf.Problem.from_scene(ctx, sc)
    xh, lam, gam, stats, status = pb.solve_subproblem(tol=1e-7, max_iter=50000, max_newton=20)
    print(f"{name}: gpu newton {stats['newton_iters']} (last r {stats['last_step']}, {stats['energy_evals']} energy "
          f"evaluations, {stats['pcg_iters']} PCG) | oracle newton {len(hist)} r {[h[1] for h in hist]}", flush=True)
    assert status == bf.BF_OK
    assert stats["newton_iters"] == len(hist) and stats["last_step"] == hist[-1][1]
    prep = oracle.prepare(sc)
    assert abs(stats["energy_initial"] - hist[0][0]) <= 1e-9 * abs(hist[0][0])
    assert abs(stats["energy_final"] - osp.energy(sc, prep, xh)) <= 1e-9 * abs(stats["energy_final"])
    assert stats["energy_final"] < stats["energy_initial"]
    # the displacement x_hat - x_hat^0 against the oracle's, in the energy norm of H at x_hat^0
    H0 = oracle.assemble(sc).H
    err = oracle.energy_norm_rel(H0, xh - sc["x_hat"], xr - sc["x_hat"])
    print(f"{name}: displacement energy-norm error {err:.2e}", flush=True)
    assert err <= 1e-4
    fixed = sc["fixed"].astype(bool)
    assert np.array_equal(xh[fixed], sc["x_hat"][fixed])
    # the update at the GPU's x_hat, against the oracle's update at that same x_hat
    lam_o, gam_o, act_o = osp.dual_update(sc, xh, Gamma=0.9)
    c = osp.constraint_values_at(sc, xh)
    margin = np.abs(c - sc["lam"] / sc["kappa"]) > 1e-9 * np.maximum(1.0, np.abs(sc["lam"] / sc["kappa"]))
    assert np.array_equal(gam[margin], gam_o[margin])
    # lambda' = lambda - kappa c: kappa times the FP64 difference of c_i
    assert np.allclose(lam[margin], lam_o[margin], rtol=1e-9, atol=1e-11 * sc["kappa"])
    assert stats["active"] == int(act_o.sum()) or not margin.all()
    assert abs(stats["max_violation"] - float(np.maximum(0.0, -c).max())) <= 1e-12


def test_outer_iterations_reach_feasibility_like_the_oracle(ctx, bf):
    """Chained subproblems (the augmented-Lagrangian outer loop): the GPU's
    constraint violation falls like the oracle's.  Each c_i is Lipschitz in
    x_hat with constant sum_a |w_a| = 2 (max norm over vertices), so the two
    violations differ by at most twice the largest vertex offset between the
    two states."""
    sc = pushed()
    pb = bf.Problem.from_scene(ctx, sc)
    so = dict(sc)
    vg, vo = [], []
    for _ in range(5):
        xh, lam, gam, stats, _ = pb.solve_subproblem(tol=1e-7, max_iter=50000, max_newton=20)
        vg.append(stats["max_violation"])
        xr, lr, gr, _ = osp.solve_subproblem(so, max_newton=20)
        vo.append(float(np.maximum(0.0, -osp.constraint_values_at(so, xr)).max()))
        so["x_hat"], so["lam"], so["gamma"] = xr, lr, gr
        # the violation the oracle computes at the GPU's own state is the GPU's, exactly
        vg_at = float(np.maximum(0.0, -osp.constraint_values_at(dict(so, x_hat=xh), xh)).max())
        assert abs(vg[-1] - vg_at) <= 1e-12
        assert abs(vg[-1] - vo[-1]) <= 2.0 * np.linalg.norm(xh - xr, axis=1).max() + 1e-15
    print(f"violation gpu {['%.2e' % v for v in vg]} oracle {['%.2e' % v for v in vo]}", flush=True)
    assert vg[-1] < 0.1 * vg[0]


def test_medium_subproblem_in_the_bench_configuration(ctx, bf):
    """The medium workload with the options the bench times (tol 1e-5, up to
    20 Newton steps): the oracle's energies and update at the GPU's states
    (its direct Newton steps would take minutes on this size; the steps
    themselves are covered by the Newton-step parity tests)."""
    sc = scenes.medium()
    pb = bf.Problem.from_scene(ctx, sc)
    xh, lam, gam, stats, status = pb.solve_subproblem(tol=1e-5, max_iter=200000, max_newton=20)
    print(f"medium: {stats}", flush=True)
    assert status == bf.BF_OK
    assert stats["last_step"] == 1.0 and stats["truncated"] == 0
    check_subproblem(sc, xh, lam, gam, stats)


def _with_x(sc, x):
    sc = dict(sc)
    sc["x"] = x
    sc["x_tilde"] = x
    sc["x_hat"] = x.copy()
    return sc


MU_CASES = {
    "tiny_rest": lambda: scenes.tiny(),
    "tiny_dilated": lambda: (lambda sc: _with_x(sc, 1.05 * sc["rest"]))(scenes.tiny()),
    # 10 % compression in z: J < 1, so the projection clamps the twist modes
    "tiny_compressed": lambda: (lambda sc: _with_x(sc, sc["rest"] * np.array([1.0, 1.0, 0.9])))(scenes.tiny()),
    "medium": scenes.medium,
}


@pytest.mark.parametrize("name", list(MU_CASES))
def test_mu_init_matches_oracle(ctx, bf, name):
    """Section 5.2's C max_i (grad^2 E)_ii: within 1e-5 relative (FP32 sums of
    the element blocks against FP64)."""
    sc = MU_CASES[name]()
    print(f"case {name}", flush=True)
    pb = bf.Problem.from_scene(ctx, sc)
    mu = pb.mu_init(0.1)
    ref = osp.mu_init(sc, 0.1)
    print(f"{name}: mu_init {mu:.9e}, oracle {ref:.9e}", flush=True)
    assert mu == pytest.approx(ref, rel=1e-5)
    assert pb.mu_init(0.2) == pytest.approx(2.0 * mu, rel=1e-15)
    # the Newton step afterwards is unaffected (it rebuilds the staged blocks at x_hat)
    p1, _, _ = pb.newton_step(tol=1e-6)
    pb2 = bf.Problem.from_scene(ctx, sc)
    p2, _, _ = pb2.newton_step(tol=1e-6)
    assert np.array_equal(p1, p2)


def test_mu_init_errors(ctx, bf):
    sc = scenes.tiny()
    pb = bf.Problem.from_scene(ctx, sc)
    for C in (0.0, -1.0, float("nan")):
        with pytest.raises(bf.BfalError):
            pb.mu_init(C)
