"""Parity at the full size of the large workload (2.25M tets, 403,155 nodes,
1.0M constraints), in the launch configuration bench.py times, against the
FP64 oracle assembled at full size (about a minute of CPU).

Bars: the merged BSR pattern and its maps bit-exact; the FP32 gradient and
blocks within 1e-5 relative, globally and per node / per block against the
summed magnitude of their terms (term_scales.py), also with the constraint set
emptied (the elastic and inertia terms alone); the returned step within twice
the FP64 solver's own error at the same tolerance plus the FP32-storage floor,
in the energy norm of the oracle's H against the oracle's reference solution
(tests/golden/large_p_ref.npy: FP64 block-Jacobi PCG to 1e-12); its residual, measured in
FP64 with the oracle's H, within 1.5e-5 of |G| (the PCG tolerance is 1e-5 on
the FP32-stored system); the FP64 stats exact to rounding."""
import json
import os

import numpy as np
import pytest

import oracle
import scenes
import term_scales
from subproblem_checks import check_subproblem

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def large():
    sc = scenes.make_scene("large")
    print("large: oracle assembly", flush=True)
    st = oracle.assemble(sc)
    return sc, st


@pytest.fixture(scope="module")
def gpu(large):
    from paper_2512_12151_amd import bfal
    import torch
    sc, _ = large
    dev = torch.device("cuda:0")
    t = {k: torch.from_numpy(np.ascontiguousarray(sc[k])).to(dev)
         for k in ("tets", "rest", "E", "nu", "rho", "fixed", "x", "x_hat", "x_tilde", "pt", "ee", "lam", "gamma")}
    torch.cuda.synchronize()
    ctx = bfal.Context(0, stream=torch.cuda.current_stream().cuda_stream)
    pb = bfal.Problem(ctx, t["tets"], t["rest"], t["E"], t["nu"], t["rho"], t["fixed"])
    pb.set_state(t["x"], t["x_hat"], t["x_tilde"], sc["dt"])
    pb.set_constraints(t["pt"], t["ee"], t["lam"], t["gamma"], sc["kappa"], sc["delta"])
    out = torch.empty((len(sc["rest"]), 3), dtype=torch.float64, device=dev)
    print("large: GPU Newton step", flush=True)
    _, stats, status = pb.newton_step(tol=1e-5, max_iter=200000, poll_every=64, check_every=4, out=out)
    torch.cuda.synchronize()
    p = out.cpu().numpy()
    res = dict(p=p, stats=stats, status=status, g=pb.gradient(), pattern=pb.pattern(), blocks=pb.blocks())
    pb.close()
    ctx.close()
    return res


@pytest.mark.timeout(600)
def test_large_pattern_bit_exact(large, gpu):
    sc, _ = large
    row_ptr, col, emap, cmap, diag = gpu["pattern"]
    r_ptr, r_col, r_emap, r_cmap, r_diag = oracle.pattern(len(sc["rest"]), sc["tets"], sc["pt"], sc["ee"])
    assert np.array_equal(row_ptr, r_ptr)
    assert np.array_equal(col, r_col)
    assert np.array_equal(emap, r_emap)
    assert np.array_equal(cmap, r_cmap)
    assert np.array_equal(diag, r_diag)


@pytest.mark.timeout(600)
def test_large_gradient_and_blocks(large, gpu):
    sc, st = large
    free = ~sc["fixed"].astype(bool)
    g = gpu["g"]
    eg = np.linalg.norm((g - st.G)[free]) / np.linalg.norm(st.G[free])
    row_ptr, col, *_ = gpu["pattern"]
    B = gpu["blocks"].astype(np.float64)
    Bref = oracle.upper_blocks(st.H, row_ptr.astype(np.int64), col)
    eb = np.linalg.norm(B - Bref) / np.linalg.norm(Bref)
    print(f"large: gradient rel {eg:.2e}, blocks rel {eb:.2e}", flush=True)
    assert eg <= 1e-5
    assert eb <= 1e-5
    assert np.all(g[~free] == 0.0)
    gs, bs = term_scales.scales(sc, st, row_ptr.astype(np.int64), col)
    rg, rb, ig, ib = term_scales.elementwise(g, st.G, B, Bref, gs, bs)
    print(f"large: element-wise gradient {rg:.2e} (node {ig}), blocks {rb:.2e} (slot {ib})", flush=True)
    assert rg <= 1e-5
    assert rb <= 1e-5


@pytest.mark.timeout(900)
def test_large_no_constraints_gradient_and_blocks():
    """The large mesh with its constraint set emptied: the elastic and inertia
    terms alone at full size, globally and element-wise within 1e-5."""
    from paper_2512_12151_amd import bfal
    sc = dict(scenes.make_scene("large"))
    z = np.zeros((0, 4), np.int32)
    sc.update(pt=z, ee=z, lam=np.zeros(0), gamma=np.zeros(0))
    ctx = bfal.Context(0)
    pb = bfal.Problem.from_scene(ctx, sc)
    print("large, no constraints: GPU assembly", flush=True)
    pb.newton_step(tol=1e-5, max_iter=0)
    g, (row_ptr, col, *_), B = pb.gradient(), pb.pattern(), pb.blocks().astype(np.float64)
    pb.close()
    ctx.close()
    print("large, no constraints: oracle assembly", flush=True)
    st = oracle.assemble(sc)
    free = ~sc["fixed"].astype(bool)
    eg = np.linalg.norm((g - st.G)[free]) / np.linalg.norm(st.G[free])
    Bref = oracle.upper_blocks(st.H, row_ptr.astype(np.int64), col)
    eb = np.linalg.norm(B - Bref) / np.linalg.norm(Bref)
    gs, bs = term_scales.scales(sc, st, row_ptr.astype(np.int64), col)
    rg, rb, _, _ = term_scales.elementwise(g, st.G, B, Bref, gs, bs)
    print(f"large, no constraints: gradient rel {eg:.2e}, blocks rel {eb:.2e}; element-wise {rg:.2e}, {rb:.2e}",
          flush=True)
    assert eg <= 1e-5 and eb <= 1e-5
    assert rg <= 1e-5 and rb <= 1e-5
    assert np.all(g[~free] == 0.0)


@pytest.mark.timeout(600)
@pytest.mark.skipif(not os.path.exists(os.path.join(GOLDEN, "large_p_ref.npy")),
                    reason="reference solution not written yet (tests/golden/make_large_reference.py)")
def test_large_solution_energy_norm(large, gpu):
    """The step against the oracle's reference solution p* in the energy norm
    of the oracle's FP64 H.  The bar adds what the two sides of the comparison
    cannot avoid: the FP64 oracle PCG's own error at the same tolerance
    (x0 = 0, |r| <= 1e-5 |b|), doubled for FP32 recurrences, and the distance
    between p* and the exact solution of the FP32-stored system (a lower bound,
    so the bar errs on the strict side); both recorded with p* by the script
    that wrote it, from the oracle alone.  Iteration counts are printed."""
    sc, st = large
    with open(os.path.join(GOLDEN, "large_p_ref.json")) as f:
        meta = json.load(f)
    assert meta["digest"] == scenes.digest(sc)
    p_ref = np.load(os.path.join(GOLDEN, "large_p_ref.npy")).astype(np.float64)
    err = oracle.energy_norm_rel(st.H, gpu["p"], p_ref)
    ref64 = meta["fp64_pcg_at_step_tol"]
    floor32 = meta["float32_storage_floor"]["energy_norm_lower_bound"]
    bar = 2.0 * ref64["energy_norm_error"] + floor32 + 1e-5
    print(f"large: energy-norm error {err:.3e} after {gpu['stats']['pcg_iters']} FP32 PCG iterations | FP64 "
          f"oracle PCG at tol {ref64['tol']:g}: {ref64['energy_norm_error']:.3e} after {ref64['iterations']} "
          f"iterations | FP32-storage floor >= {floor32:.2e} | bar {bar:.3e} | p* storage "
          f"{meta['float32_storage_energy_norm_error']:.1e}", flush=True)
    assert err <= bar


@pytest.mark.timeout(600)
def test_large_solution_residual_and_stats(large, gpu):
    sc, st = large
    p, stats = gpu["p"], gpu["stats"]
    assert gpu["status"] == 0
    r = st.H @ p.ravel() + st.G.ravel()
    rel = np.linalg.norm(r) / np.linalg.norm(st.G)
    print(f"large: {stats['pcg_iters']} PCG iterations, solver residual {stats['rel_residual']:.3e}, "
          f"FP64 residual with the oracle's H {rel:.3e}", flush=True)
    assert stats["rel_residual"] <= 1e-5
    assert rel <= 1.5e-5
    assert np.all(p[sc["fixed"].astype(bool)] == 0.0)
    viol = float(np.maximum(0.0, -st.c).max())
    assert abs(stats["max_violation"] - viol) <= 1e-12 * max(1.0, viol)
    assert np.isclose(stats["newton_inf_over_h"], np.abs(p).max() / sc["dt"], rtol=1e-12)


@pytest.mark.timeout(600)
def test_large_subproblem_energy_and_update(large):
    """Four Newton steps of SolveSubproblem at full size (damped: the line
    search cuts the first steps to r ~ 1/64 here), then the multiplier update:
    the oracle's FP64 energies and update at the GPU's states."""
    from paper_2512_12151_amd import bfal
    sc, _ = large
    ctx = bfal.Context(0)
    pb = bfal.Problem.from_scene(ctx, sc)
    print("large: GPU subproblem", flush=True)
    xh, lam, gam, stats, status = pb.solve_subproblem(tol=1e-5, max_iter=200000, max_newton=4)
    pb.close()
    ctx.close()
    print(f"large subproblem: status {status} {stats}", flush=True)
    assert status in (bfal.BF_OK, bfal.BF_WARN_PCG_MAXITER)
    assert stats["newton_iters"] == 4 and 0.0 < stats["last_step"] < 1.0
    check_subproblem(sc, xh, lam, gam, stats)


@pytest.mark.timeout(600)
def test_large_mu_init(large):
    """Section 5.2's penalty estimate at the large workload's x (the stack
    compressed 40 % in z, so the projection is active in many tets): within
    1e-5 relative of the oracle's FP64 value."""
    from oracle import subproblem as osp
    from paper_2512_12151_amd import bfal
    sc, _ = large
    ctx = bfal.Context(0)
    pb = bfal.Problem.from_scene(ctx, sc)
    mu = pb.mu_init(0.1)
    pb.close()
    ctx.close()
    print("large: oracle mu_init", flush=True)
    ref = osp.mu_init(sc, 0.1)
    print(f"large: mu_init {mu:.9e}, oracle {ref:.9e} (the workload's kappa {sc['kappa']:.0e})", flush=True)
    assert mu == pytest.approx(ref, rel=1e-5)
