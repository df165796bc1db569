"""Per-tet materials (Table 2: Neo-Hookean, stable Neo-Hookean, corotated
linear) on the GPU against the FP64 oracle, through the C-ABI.

States: the shifted tiny stack, all stable Neo-Hookean, all corotated, mixed
with Neo-Hookean (upper cube the other material) or all three cycling per tet,
at the generator's 1 % noise and under three large deformations that reach
every branch of the element kernel's projection: the lower cube stretched 1.8x
in z (J up to 1.89; stable Neo-Hookean: q = J (lam (J-1) - mu) > 0, the 3x3
scaling Hessian is clamped), compressed to 0.6x (J down to 0.57: r + q =
J (lam (2J - 1) - mu) < 0, clamped as well; corotated: the twist modes
(Psi_i + Psi_j) / (S_i + S_j) turn negative and are clamped) and sheared by 0.5.

Bars, as for Neo-Hookean: the FP32 gradient and the assembled blocks within
1e-5 relative, the FP64 energy within 1e-9 relative, the Newton direction
within 1e-4 in the energy norm of the oracle's H, and SolveSubproblem by the
shared subproblem checks plus its displacement within 1e-4 in that norm."""
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


def deformed(material, kind):
    sc = dict(scenes.tiny(lateral=(0.37, 0.21), material=material))
    xh = sc["x_hat"].copy()
    lower = sc["rest"][:, 2] <= 1.0
    if kind == "stretch":
        sc["dt"] = 1.0
        xh[lower, 2] = sc["rest"][lower, 2] * 1.8
        xh[~lower, 2] = sc["rest"][~lower, 2] + 0.8
    elif kind == "compress":
        xh[lower, 2] = sc["rest"][lower, 2] * 0.6
        xh[~lower, 2] = sc["rest"][~lower, 2] - 0.4
    elif kind == "shear":
        xh[:, 0] += 0.5 * sc["rest"][:, 2]
    sc["x_hat"] = np.where(sc["fixed"][:, None] == 1, sc["x"], xh)
    return sc


CASES = [(m, k) for m in ("snh", "mixed", "cor", "mixed_cor", "all3") for k in ("noise", "stretch", "compress", "shear")]


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("material,kind", CASES)
def test_gradient_blocks_energy(ctx, bf, material, kind):
    print(f"case {material}/{kind}", flush=True)
    sc = deformed(material, kind)
    st = oracle.assemble(sc)
    pb = bf.Problem.from_scene(ctx, sc)
    p, stats, status = pb.newton_step(tol=1e-7, max_iter=50000)
    assert status == bf.BF_OK
    free = ~sc["fixed"].astype(bool)
    g = pb.gradient()
    eg = rel(g[free], st.G[free])
    row_ptr, col, *_ = pb.pattern()
    B = pb.blocks().astype(np.float64)
    eb = rel(B, oracle.upper_blocks(st.H, row_ptr.astype(np.int64), col))
    L, inv = pb.energy()
    Lref = oracle.total_energy(sc, oracle.prepare(sc), sc["x_hat"])
    ep = oracle.energy_norm_rel(st.H, p, oracle.solve_reference(st.H, st.G))
    print(f"{material}/{kind}: gradient {eg:.2e} blocks {eb:.2e} energy {abs(L - Lref) / abs(Lref):.2e} "
          f"direction {ep:.2e} ({stats['pcg_iters']} PCG)", flush=True)
    assert eg <= 1e-5 and eb <= 1e-5
    assert not inv and abs(L - Lref) <= 1e-9 * abs(Lref)
    assert ep <= 1e-4


@pytest.mark.parametrize("material,kind", [("snh", "stretch"), ("mixed", "stretch"), ("snh", "compress"),
                                           ("cor", "compress"), ("mixed_cor", "stretch"), ("all3", "stretch")])
def test_subproblem(ctx, bf, material, kind):
    print(f"case {material}/{kind}", flush=True)
    sc = deformed(material, kind)
    xr, lam_r, gam_r, hist = osp.solve_subproblem(sc, max_newton=20)
    pb = bf.Problem.from_scene(ctx, sc)
    xh, lam, gam, stats, status = pb.solve_subproblem(tol=1e-7, max_iter=50000, max_newton=20)
    print(f"{material}/{kind}: gpu newton {stats['newton_iters']} r {stats['last_step']} | oracle "
          f"{len(hist)} r {[h[1] for h in hist]}", flush=True)
    assert status == bf.BF_OK
    assert stats["newton_iters"] == len(hist) and stats["last_step"] == hist[-1][1]
    check_subproblem(sc, xh, lam, gam, stats)
    err = oracle.energy_norm_rel(oracle.assemble(sc).H, xh - sc["x_hat"], xr - sc["x_hat"])
    print(f"{material}/{kind}: displacement energy-norm error {err:.2e}", flush=True)
    assert err <= 1e-4


def test_neo_hookean_code_matches_no_material_array(ctx, bf):
    """An explicit all-zero material array is the default path, bit for bit."""
    sc = deformed(None, "stretch")
    a = bf.Problem.from_scene(ctx, sc)
    pa, _, _ = a.newton_step(tol=1e-7)
    sc0 = dict(sc, material=np.zeros(len(sc["tets"]), dtype=np.int32))
    b = bf.Problem.from_scene(ctx, sc0)
    pb_, _, _ = b.newton_step(tol=1e-7)
    assert np.array_equal(a.gradient(), b.gradient()) and np.array_equal(a.blocks(), b.blocks())
    assert np.array_equal(pa, pb_)
    assert a.energy() == b.energy()


@pytest.mark.parametrize("material", ["mixed", "all3"])
def test_mu_init_materials(ctx, bf, material):
    """Section 5.2's mu_init on meshes of several materials (at x, the start state)."""
    sc = deformed(material, "stretch")
    sc["x"] = sc["x_hat"].copy()
    pb = bf.Problem.from_scene(ctx, sc)
    m = pb.mu_init(0.1)
    ref = osp.mu_init(sc, 0.1)
    print(f"mu_init {m:.9e} oracle {ref:.9e}", flush=True)
    assert m == pytest.approx(ref, rel=1e-5)   # FP32 sums of the element blocks against FP64


def test_invalid_material_code_rejected(ctx, bf):
    sc = dict(scenes.tiny(material="snh"))
    sc["material"] = sc["material"].copy()
    sc["material"][3] = 3
    with pytest.raises(bf.BfalError) as e:
        bf.Problem.from_scene(ctx, sc)
    assert e.value.status == -1   # BF_ERR_INVALID_ARG
