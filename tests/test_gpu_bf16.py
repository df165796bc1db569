"""BF16 block storage inside FP32/FP64 iterative refinement, against the FP64
oracle (the precision variant of the medium workload).

The scaled blocks are rounded to BF16 (nearest even) for the inner PCG; the
outer loop (flexible CG on the FP32-stored system) keeps the solution in FP64
and forms the residual in FP64.  Bars: the refined solution within 1e-4 relative in
the oracle's FP64 energy norm of the direct solution, and the FP64 residual
reported by the library at or below the requested 1e-6.  The energy-norm error
of every sweep is printed beside the FP32 baseline at the same tolerance."""
import numpy as np
import pytest

import oracle
import scenes

pytestmark = pytest.mark.gpu

_cache = {}


def ref(name):
    if name not in _cache:
        sc = scenes.medium() if name == "medium" else scenes.tiny(lateral=(0.37, 0.21))
        st = oracle.assemble(sc)
        _cache[name] = (sc, st, oracle.solve_reference(st.H, st.G))
    return _cache[name]


@pytest.fixture(scope="module")
def bf():
    from paper_2512_12151_amd import bfal
    return bfal


@pytest.fixture(scope="module")
def ctx(bf):
    return bf.Context(0)


@pytest.mark.parametrize("name", ["tiny_shifted", "medium"])
def test_bf16_refinement_matches_fp64(ctx, bf, name):
    sc, st, p_ref = ref(name)
    print(f"case {name}", flush=True)
    pb = bf.Problem.from_scene(ctx, sc)
    p, stats, status = pb.newton_step(tol=0.3, refine_tol=1e-6, precision=bf.BF_PREC_BF16_REFINE,
                                      max_iter=50000)
    assert status == bf.BF_OK
    err = oracle.energy_norm_rel(st.H, p, p_ref)
    p32, s32, _ = pb.newton_step(tol=1e-6, max_iter=50000)
    err32 = oracle.energy_norm_rel(st.H, p32, p_ref)
    res = stats["sweep_rel_residual"]
    print(f"{name}: bf16+refine sweeps={stats['refine_sweeps']} inner iters={stats['pcg_iters']} err={err:.3e} "
          f"residuals={['%.2e' % r for r in res]} | fp32 tol 1e-6 iters={s32['pcg_iters']} err={err32:.3e}",
          flush=True)
    assert stats["rel_residual"] <= 1e-6
    assert res[0] == pytest.approx(1.0, rel=1e-6)
    assert err <= 1e-4
    assert np.all(p[sc["fixed"].astype(bool)] == 0.0)
    # the true FP64 residual with the oracle's H is bounded by the FP32 storage of H
    r = st.H @ p.ravel() + st.G.ravel()
    assert np.linalg.norm(r) <= 1e-4 * np.linalg.norm(st.G)


def test_bf16_error_per_sweep(ctx, bf):
    """Energy-norm error after s sweeps (max_sweeps = s): it falls with the
    sweeps and ends inside the bar; the FP32 PCG at the same final residual is
    printed beside it."""
    sc, st, p_ref = ref("medium")
    pb = bf.Problem.from_scene(ctx, sc)
    opts = dict(tol=0.3, refine_tol=1e-6, precision=bf.BF_PREC_BF16_REFINE, max_iter=50000)
    _, full, _ = pb.newton_step(**opts)
    n = full["refine_sweeps"]
    errs = []
    for s in sorted(set([1, 2, 4, 8, 16, 32, n]) & set(range(1, n + 1))):
        p, stats, status = pb.newton_step(max_sweeps=s, **opts)
        errs.append(oracle.energy_norm_rel(st.H, p, p_ref))
        print(f"medium bf16 sweep {s}: rel residual {stats['rel_residual']:.3e} inner iterations "
              f"{stats['pcg_iters']} energy-norm error {errs[-1]:.3e}", flush=True)
    p32, s32, _ = pb.newton_step(tol=1e-6, max_iter=50000)
    print(f"medium fp32 tol 1e-6: iterations {s32['pcg_iters']} energy-norm error "
          f"{oracle.energy_norm_rel(st.H, p32, p_ref):.3e}", flush=True)
    assert errs[-1] <= 1e-4
    assert errs[-1] < errs[0]
