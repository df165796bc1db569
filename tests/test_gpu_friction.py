"""Semi-implicit friction (Appendix A) on the GPU against the FP64 oracle,
through the C-ABI.

Sliding state: the shifted tiny stack with multipliers that press every
contact, the friction set captured at x (mu_f = 0.5, eps_v h = 5 mm, so that
the 1 % noise of x_hat puts contacts on both sides of the smoothing
threshold) and the upper cube pushed sideways.  Bars as for the frictionless
step: the pattern bit-exact, G and blocks within 1e-5 relative, the FP64
energy within 1e-9, the Newton direction within 1e-4 in the energy norm and
the subproblem's Newton loop like the oracle's.

Time step: the thrown cube with a lateral velocity of 0.2 m/s; the step after
landing, from the oracle's first step, with friction captured from its
contacts (mu_f = 0.5, eps_v = 1e-3 as in Table 2).  The bars are those of the
frictionless time-step test (same iterations and active set, state within
1e-3 of the displacement), and friction must slow the lateral motion as the
oracle's does."""
import numpy as np
import pytest

import oracle
from oracle import friction as ofr
from oracle import subproblem as osp
from oracle import timestep
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


MU_F, EPS_V = 0.5, 0.5


def sliding(seed=1):
    """(scene without friction, the same with the oracle's friction set)."""
    sc = dict(scenes.tiny(lateral=(0.37, 0.21)))
    sc["lam"] = np.random.default_rng(seed).uniform(20.0, 60.0, size=len(sc["lam"]))
    f = ofr.capture(sc, MU_F, EPS_V)
    upper = sc["rest"][:, 2] > 1.0
    xh = sc["x_hat"].copy()
    xh[upper, 0] += np.linspace(0.0, 3e-4, upper.sum())
    sc["x_hat"] = xh
    return sc, dict(sc, friction=f)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_step_with_friction_matches_oracle(ctx, bf):
    sc, scf = sliding()
    st = oracle.assemble(scf)
    pb = bf.Problem.from_scene(ctx, sc)
    pb.set_friction(MU_F, EPS_V)
    p, stats, status = pb.newton_step(tol=1e-7, max_iter=50000)
    assert status == bf.BF_OK
    row_ptr, col, emap, cmap, diag = pb.pattern()
    r_ptr, r_col, r_emap, _, r_diag = oracle.pattern(len(sc["rest"]), sc["tets"], sc["pt"], sc["ee"])
    assert np.array_equal(row_ptr, r_ptr) and np.array_equal(col, r_col)
    free = ~sc["fixed"].astype(bool)
    eg = rel(pb.gradient()[free], st.G[free])
    eb = rel(pb.blocks().astype(np.float64), oracle.upper_blocks(st.H, row_ptr.astype(np.int64), col))
    L, inv = pb.energy()
    Lref = oracle.total_energy(scf, oracle.prepare(scf), scf["x_hat"])
    ep = oracle.energy_norm_rel(st.H, p, oracle.solve_reference(st.H, st.G))
    # the friction terms are a visible part of G
    g0 = oracle.assemble(sc).G
    print(f"friction: |G_f| / |G| {rel(st.G[free], g0[free]):.2e}; gradient {eg:.2e} blocks {eb:.2e} energy "
          f"{abs(L - Lref) / abs(Lref):.2e} direction {ep:.2e}", flush=True)
    assert rel(st.G[free], g0[free]) > 1e-3
    assert eg <= 1e-5 and eb <= 1e-5
    assert not inv and abs(L - Lref) <= 1e-9 * abs(Lref)
    assert ep <= 1e-4
    # mu_f = 0 clears the set: the frictionless step again
    pb.set_friction(0.0)
    pb.newton_step(tol=1e-7)
    assert rel(pb.gradient()[free], g0[free]) <= 1e-5


def test_friction_set_outlives_a_constraint_change(ctx, bf):
    """After the capture, a new constraint set (every other constraint) keeps
    the captured friction contacts: their stencils stay in the pattern."""
    sc, scf = sliding(2)
    pb = bf.Problem.from_scene(ctx, sc)
    pb.set_friction(MU_F, EPS_V)
    keep_pt, keep_ee = sc["pt"][::2], sc["ee"][::2]
    n_pt = len(sc["pt"])
    lam = np.concatenate([sc["lam"][:n_pt][::2], sc["lam"][n_pt:][::2]])
    gam = np.concatenate([sc["gamma"][:n_pt][::2], sc["gamma"][n_pt:][::2]])
    pb.set_constraints(keep_pt, keep_ee, lam, gam, sc["kappa"], sc["delta"])
    p, _, status = pb.newton_step(tol=1e-7, max_iter=50000)
    assert status == bf.BF_OK
    sub = dict(scf, pt=keep_pt, ee=keep_ee, lam=lam, gamma=gam)
    st = oracle.assemble(sub)
    row_ptr, col, *_ = pb.pattern()
    r_ptr, r_col, *_ = oracle.pattern(len(sc["rest"]), sc["tets"], np.concatenate([keep_pt, sc["pt"]]),
                                      np.concatenate([keep_ee, sc["ee"]]))
    assert np.array_equal(row_ptr, r_ptr) and np.array_equal(col, r_col)
    free = ~sc["fixed"].astype(bool)
    assert rel(pb.gradient()[free], st.G[free]) <= 1e-5
    assert rel(pb.blocks().astype(np.float64), oracle.upper_blocks(st.H, row_ptr.astype(np.int64), col)) <= 1e-5
    L, _ = pb.energy()
    Lref = oracle.total_energy(sub, oracle.prepare(sub), sub["x_hat"])
    assert abs(L - Lref) <= 1e-9 * abs(Lref)
    assert oracle.energy_norm_rel(st.H, p, oracle.solve_reference(st.H, st.G)) <= 1e-4


@pytest.mark.parametrize("eps_v", [5.0, 1.0])
def test_subproblem_with_friction(ctx, bf, eps_v):
    """One full Newton step from a sideways push of 3 mm: eps_v h = 5 cm keeps
    every contact sticking, eps_v h = 1 cm lets 3 % of them cross into sliding
    during the step.  (Where x_hat starts far outside the smoothing band the
    loop crawls through many line-searched steps on both sides, and their end
    states, taken at the first full step, depend on the path.)"""
    slide = 3e-3
    sc = dict(scenes.tiny(lateral=(0.37, 0.21)))
    sc["lam"] = np.random.default_rng(3).uniform(20.0, 60.0, size=len(sc["lam"]))
    f = ofr.capture(sc, MU_F, eps_v)
    upper = sc["rest"][:, 2] > 1.0
    xh0 = sc["x_hat"].copy()
    xh0[upper, 0] += np.linspace(0.0, slide, upper.sum())
    sc["x_hat"] = xh0
    scf = dict(sc, friction=f)
    xr, lam_r, gam_r, hist = osp.solve_subproblem(scf, max_newton=20)
    pb = bf.Problem.from_scene(ctx, sc)
    pb.set_friction(MU_F, eps_v)
    xh, lam, gam, stats, status = pb.solve_subproblem(tol=1e-7, max_iter=50000, max_newton=20)
    print(f"friction subproblem eps_v {eps_v}: gpu newton {stats['newton_iters']} r {stats['last_step']} | oracle "
          f"{len(hist)} r {[h[1] for h in hist]}", flush=True)
    assert status == bf.BF_OK
    assert stats["newton_iters"] == len(hist) and stats["last_step"] == hist[-1][1]
    check_subproblem(scf, xh, lam, gam, stats)
    err = oracle.energy_norm_rel(oracle.assemble(scf).H, xh - scf["x_hat"], xr - scf["x_hat"])
    Lr = hist[-1][2]
    print(f"friction subproblem eps_v {eps_v}: displacement energy-norm error {err:.2e}, final energy "
          f"{stats['energy_final']:.12e} oracle {Lr:.12e}", flush=True)
    assert len(hist) == 1 and err <= 1e-4


def _landed():
    """The thrown cube (jittered, lateral 0.2 m/s) after the oracle's first step."""
    sc = dict(scenes.falling_cubes(jitter=1e-5))
    N, h = len(sc["x"]), sc["dt"]
    sc["x_tilde"] = sc["x_tilde"].copy()
    sc["x_tilde"][N // 2:, 0] += h * 0.2
    x1, v1, (pt, ee, lam, gam), info = timestep.time_step(sc, mu_f=0.5)
    return dict(sc, x=x1, x_hat=x1.copy(), x_tilde=x1 + h * v1, pt=pt, ee=ee, lam=lam, gamma=gam,
                kappa=info["kappa"], delta=info["delta"])


def test_time_step_with_friction_matches_oracle(ctx, bf):
    sc2 = _landed()
    N = len(sc2["x"])
    up = np.arange(N) >= N // 2
    res = {}
    for mu in (0.0, 0.5):
        xo, vo, (pto, eeo, lamo, gamo), info = timestep.time_step(sc2, mu_f=mu, eps_v=1e-3)
        pb = bf.Problem.from_scene(ctx, sc2)
        x, v, st, status = pb.time_step(tol=1e-9, mu_f=mu, eps_v=1e-3, k_min=2)
        print(f"mu_f {mu}: gpu {st['outer_iters']} iterations, vx {v[up, 0].mean():.6f} | oracle {info['outer']} "
              f"alphas {info['alphas']}, vx {vo[up, 0].mean():.6f}", flush=True)
        assert status == bf.BF_OK
        assert st["outer_iters"] == info["outer"]
        disp = np.abs(xo - sc2["x"]).max()
        err = np.abs(x - xo).max()
        print(f"mu_f {mu}: max |x - x_oracle| {err:.3e} of displacement {disp:.3e}", flush=True)
        assert err <= 1e-3 * disp
        pt, ee, lam, gam = pb.constraints()
        assert np.array_equal(pt, pto) and np.array_equal(ee, eeo)
        res[mu] = (v[up, 0].mean(), vo[up, 0].mean())
    # friction takes lateral speed off, as much as in the oracle
    dg, do = res[0.0][0] - res[0.5][0], res[0.0][1] - res[0.5][1]
    print(f"lateral slow-down: gpu {dg:.6f} oracle {do:.6f}", flush=True)
    assert do > 0.01 and abs(dg - do) <= 1e-2 * do


def test_set_friction_errors(ctx, bf):
    sc, _ = sliding()
    pb = bf.Problem.from_scene(ctx, sc)
    for mu, ev in ((-1.0, 1e-3), (np.inf, 1e-3), (0.5, 0.0), (0.5, np.nan)):
        with pytest.raises(bf.BfalError) as e:
            pb.set_friction(mu, ev)
        assert e.value.status == -1   # BF_ERR_INVALID_ARG


def test_friction_without_constraints_and_determinism(ctx, bf):
    """Every constraint removed after the capture: all friction contacts keep
    stencils of their own (the constraint table is empty).  With the matched
    set, two steps are bitwise equal (the matching keeps the assembly order)."""
    sc, scf = sliding(5)
    pb = bf.Problem.from_scene(ctx, sc)
    pb.set_friction(MU_F, EPS_V)
    p1, s1, _ = pb.newton_step(tol=1e-7)
    g1, b1 = pb.gradient(), pb.blocks()
    p2, s2, _ = pb.newton_step(tol=1e-7)
    assert np.array_equal(p1, p2) and np.array_equal(g1, pb.gradient()) and np.array_equal(b1, pb.blocks())
    assert s1["pcg_iters"] == s2["pcg_iters"]
    empty = np.zeros((0, 4), dtype=np.int32)
    pb.set_constraints(empty, empty, np.zeros(0), np.zeros(0), sc["kappa"], sc["delta"])
    p, _, status = pb.newton_step(tol=1e-7, max_iter=50000)
    assert status == bf.BF_OK
    sub = dict(scf, pt=empty, ee=empty, lam=np.zeros(0), gamma=np.zeros(0))
    st = oracle.assemble(sub)
    row_ptr, col, *_ = pb.pattern()
    r_ptr, r_col, *_ = oracle.pattern(len(sc["rest"]), sc["tets"], sc["pt"], sc["ee"])
    assert np.array_equal(row_ptr, r_ptr) and np.array_equal(col, r_col)
    free = ~sc["fixed"].astype(bool)
    assert rel(pb.gradient()[free], st.G[free]) <= 1e-5
    assert rel(pb.blocks().astype(np.float64), oracle.upper_blocks(st.H, row_ptr.astype(np.int64), col)) <= 1e-5
    L, _ = pb.energy()
    Lref = oracle.total_energy(sub, oracle.prepare(sub), sub["x_hat"])
    assert abs(L - Lref) <= 1e-9 * abs(Lref)
    assert oracle.energy_norm_rel(st.H, p, oracle.solve_reference(st.H, st.G)) <= 1e-4


@pytest.mark.parametrize("mu_f", [0.0, 0.3, 0.6])
def test_block_on_slope(ctx, bf, mu_f):
    """Section 6's cubes on a slope (incline arctan 0.5, gravity tilted instead
    of the ground), through the GPU's time steps with friction (K_min = 6,
    mu_init at the first step, eps_v = 1e-3): below tan(theta) = 0.5 the block
    slides at the analytic g (sin - mu_f cos) once the contact force has settled
    at the weight (from the sixth step), within 1 % without friction and 3 %
    with it; above it (mu_f = 0.6) the block stops: after 20 steps it moves at
    under 1 cm/s, against 0.26 m/s at mu_f = 0.3 after 12."""
    sc = scenes.slope()
    N, h, g = len(sc["x"]), sc["dt"], sc["gravity"]
    up = np.arange(N) >= N // 2
    pb = bf.Problem.from_scene(ctx, sc)
    x, v = sc["x"].copy(), np.zeros_like(sc["x"])
    steps = 20 if mu_f > 0.5 else 12
    vs = []
    for step in range(steps):
        xt = x + h * v
        xt[up] += h * h * g
        pb.set_state(x, x.copy(), xt, h)
        x, v, st, status = pb.time_step(tol=1e-7, k_min=6, mu_f=mu_f, eps_v=1e-3,
                                        mu_init_c=0.1 if step == 0 else 0.0)
        assert status == bf.BF_OK
        vs.append(v[up, 0].mean())
    th = np.arctan(0.5)
    print(f"slope mu_f {mu_f}: v {np.round(vs, 4)}", flush=True)
    if mu_f < 0.5:
        a = (vs[-1] - vs[5]) / (h * (len(vs) - 6))
        a_th = 9.8 * (np.sin(th) - mu_f * np.cos(th))
        print(f"slope mu_f {mu_f}: acceleration {a:.4f}, analytic {a_th:.4f}", flush=True)
        assert a == pytest.approx(a_th, rel=0.01 if mu_f == 0.0 else 0.03)
    else:
        assert abs(vs[-1]) < 0.01 and max(vs) < 0.1


def test_momentum_conservation_with_friction(ctx, bf):
    """Section 6's momentum conservation: two free cubes (no fixed node, no
    gravity), the upper thrown at (0.2, 0, -0.5) m/s onto the lower, five time
    steps with friction.  Contact and friction forces act through weights
    that sum to zero, and every energy is translation invariant, so the
    incremental potential's gradient sums to M (x - x_tilde) over the nodes:
    each Newton step changes the total momentum by the node sum of its linear
    residual over h.  The PCG solves to 1e-9, and the FP32 blocks keep the
    translation nullspace (the node sums of each block row vanish) only to
    their 6e-8 rounding, so the momentum drifts by ~1e-7 of |P| per step
    (measured 1.05e-7 at most); the bar is 1e-6 over the five steps."""
    sc = dict(scenes.falling_cubes(jitter=1e-5))
    N, h = len(sc["x"]), sc["dt"]
    up = np.arange(N) >= N // 2
    sc["fixed"] = np.zeros(N, dtype=np.uint8)
    m = oracle.prepare(sc).mass
    pb = bf.Problem.from_scene(ctx, sc)
    x, v = sc["x"].copy(), np.zeros_like(sc["x"])
    v[up] = [0.2, 0.0, -0.5]
    P0 = (m[:, None] * v).sum(0)
    errs = []
    for step in range(5):
        pb.set_state(x, x.copy(), x + h * v, h)
        x, v, st, status = pb.time_step(tol=1e-9, max_iter=100000, k_min=6, mu_f=0.5, eps_v=1e-3)
        assert status == bf.BF_OK
        P = (m[:, None] * v).sum(0)
        errs.append(float(np.abs(P - P0).max() / np.abs(P0).max()))
        print(f"momentum step {step}: P {P}, relative change {errs[-1]:.2e}, lower cube v {v[~up].mean(0)}",
              flush=True)
    assert v[~up].mean(0)[0] > 0.005          # friction dragged the lower cube along
    assert max(errs) <= 1e-6


def test_friction_stiffer_than_fp32_blocks_reports_not_spd(ctx, bf):
    """The documented limit of FP32 blocks: a sticking stiffness 2 coef /
    (eps_v h) = 1e11 against nodal masses of a few kg leaves FP32 rounding
    residues (~6e-8 x 4 x 1e11) far above the smallest stiffness of the
    assembled matrix, which is then indefinite.  The step must say so
    (BF_ERR_NOT_SPD from a diagonal block's factorization or a PCG breakdown)
    instead of returning a direction; the same problem with friction off
    still solves.  The computation is bitwise deterministic, so the outcome
    is the same on every run."""
    sc, _ = sliding(3)
    sc = dict(sc, lam=np.full(len(sc["lam"]), 1e6))
    pb = bf.Problem.from_scene(ctx, sc)
    pb.set_friction(0.5, 1e-3)
    with pytest.raises(bf.BfalError) as e:
        pb.newton_step(tol=1e-7, max_iter=20000)
    assert e.value.status == -6   # BF_ERR_NOT_SPD
    pb.set_friction(0.0)
    _, _, status = pb.newton_step(tol=1e-7, max_iter=20000)
    assert status in (bf.BF_OK, bf.BF_WARN_PCG_MAXITER)
