"""Pins of the oracle's assembled G and H, its DBC handling, its pattern and
maps, and its reference solves."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import scenes

RNG = np.random.default_rng(5)


def free(scene):
    s = dict(scene)
    s["fixed"] = np.zeros_like(scene["fixed"])
    return s


@pytest.fixture(scope="module")
def tiny():
    return scenes.tiny()


@pytest.fixture(scope="module")
def shifted():
    return scenes.tiny(lateral=(0.37, 0.21))


@pytest.mark.parametrize("which", ["tiny", "shifted"])
def test_gradient_is_fd_of_total_energy(which, tiny, shifted):
    sc = free(tiny if which == "tiny" else shifted)
    st = oracle.assemble(sc)
    for _ in range(3):
        v = RNG.normal(size=sc["x_hat"].shape)
        eps = 1e-7
        Lp = oracle.total_energy(sc, st, sc["x_hat"] + eps * v)
        Lm = oracle.total_energy(sc, st, sc["x_hat"] - eps * v)
        fd = (Lp - Lm) / (2 * eps)
        an = float(np.sum(st.G * v))
        assert abs(fd - an) <= 1e-6 * (abs(an) + np.abs(st.G).sum() * 1e-3)


def test_dbc_gradient_and_rows(tiny):
    st = oracle.assemble(tiny)
    fx = tiny["fixed"].astype(bool)
    assert fx.sum() == 25
    assert np.all(st.G[fx] == 0.0)
    H = st.H.tocsr()
    fd = np.flatnonzero(np.repeat(fx, 3))
    Hd = H.toarray()
    for r in fd:
        assert set(np.flatnonzero(Hd[r])) == {r}
        assert set(np.flatnonzero(Hd[:, r])) == {r}
        assert Hd[r, r] > 0
    p = oracle.solve_direct(st.H, st.G)
    assert np.all(p[fx] == 0.0)


def test_translation_nullspace_of_stiffness_and_contact(shifted):
    sc = free(shifted)
    st = oracle.assemble(sc)
    M = sp.diags(np.repeat(st.mass, 3))
    K = (st.H - M).tocsr()
    for t in np.eye(3):
        v = np.tile(t, len(st.mass))
        assert np.abs(K @ v).max() <= 1e-10 * abs(K).max()


def test_rest_state_without_constraints_has_zero_gradient(tiny):
    sc = free(tiny)
    sc["x_hat"] = sc["rest"].copy()
    sc["x_tilde"] = sc["rest"].copy()
    sc["x"] = sc["rest"].copy()
    sc["pt"] = np.zeros((0, 4), np.int32)
    sc["ee"] = np.zeros((0, 4), np.int32)
    sc["lam"] = np.zeros(0)
    sc["gamma"] = np.zeros(0)
    st = oracle.assemble(sc)
    assert np.abs(st.G).max() <= 1e-9


def test_al_energy_c1_and_gradient_factor():
    mu, lam = 1e4, 37.0
    c = np.linspace(-0.02, 0.02, 4001)
    c = np.concatenate([c, [lam / mu]])
    gam = np.full_like(c, 0.7)
    ones = np.ones_like(c)
    e = oracle.al_energy(c, lam * ones, gam, mu)
    gfac, hfac = oracle.al_terms(c, lam * ones, gam, mu, None, None)
    h = 1e-8
    fd = (oracle.al_energy(c + h, lam * ones, gam, mu) - oracle.al_energy(c - h, lam * ones, gam, mu)) / (2 * h)
    assert np.allclose(fd, gfac, atol=1e-4)
    # closed form of the slack-eliminated penalty: min(mu c - lambda, 0) * gamma
    assert np.allclose(gfac, gam * np.minimum(mu * c - lam, 0.0), atol=1e-9)
    assert np.allclose(hfac, mu * gam)
    # value continuity at mu c = lambda
    assert np.isclose(oracle.al_energy(np.array([lam / mu]), np.array([lam]), np.array([1.0]), mu)[0],
                      -lam ** 2 / (2 * mu))


def _brute_pattern(N, stencils):
    S = set((v, v) for v in range(N))
    for st in stencils:
        for row in st:
            for a in range(4):
                for b in range(4):
                    if a != b:
                        S.add((min(row[a], row[b]), max(row[a], row[b])))
    return sorted(S)


@pytest.mark.parametrize("case", ["one_tet", "two_tets", "tiny", "shifted"])
def test_pattern_against_brute_force(case, tiny, shifted):
    if case == "one_tet":
        N, T, C = 4, np.array([[0, 1, 2, 3]]), np.zeros((0, 4), np.int64)
    elif case == "two_tets":
        N, T, C = 5, np.array([[0, 1, 2, 3], [4, 3, 2, 1]]), np.array([[4, 0, 1, 2]])
    else:
        sc = tiny if case == "tiny" else shifted
        N, T, C = len(sc["rest"]), sc["tets"], np.concatenate([sc["pt"], sc["ee"]])
    row_ptr, col, emap, cmap, diag = oracle.pattern(N, T, C, C[:0])
    want = _brute_pattern(N, [T, C])
    got = [(r, int(c)) for r in range(N) for c in col[row_ptr[r]:row_ptr[r + 1]]]
    assert got == want
    rows = np.repeat(np.arange(N), np.diff(row_ptr))
    for S, mp in ((np.asarray(T), emap), (np.asarray(C), cmap)):
        for k, (a, b) in enumerate(oracle.PAIRS):
            lo = np.minimum(S[:, a], S[:, b])
            hi = np.maximum(S[:, a], S[:, b])
            assert np.array_equal(rows[mp[:, k]], lo) and np.array_equal(col[mp[:, k]], hi)
    assert np.array_equal(rows[diag], np.arange(N)) and np.array_equal(col[diag], np.arange(N))


def kuhn_box_edges(nx, ny, nz):
    axis = nx * (ny + 1) * (nz + 1) + (nx + 1) * ny * (nz + 1) + (nx + 1) * (ny + 1) * nz
    faces = nx * ny * (nz + 1) + nx * (ny + 1) * nz + (nx + 1) * ny * nz
    return axis + faces + nx * ny * nz


@pytest.mark.parametrize("dims", [(4, 4, 4), (10, 10, 10), (5, 3, 2)])
def test_elastic_block_count_matches_kuhn_edge_formula(dims):
    X, T = scenes.kuhn_box(*dims, 0.1)
    row_ptr, col, *_ = oracle.pattern(len(X), T, np.zeros((0, 4), np.int64), np.zeros((0, 4), np.int64))
    assert row_ptr[-1] == len(X) + kuhn_box_edges(*dims)


def test_config_block_counts():
    # elastic upper blocks before contacts: 1,458 (tiny), 185,220 (medium), 3,111,305 (large)
    assert 2 * (125 + kuhn_box_edges(4, 4, 4)) == 1458
    assert 20 * (1331 + kuhn_box_edges(10, 10, 10)) == 185220
    assert 5 * (51 * 51 * 31 + kuhn_box_edges(50, 50, 30)) == 3111305


def test_direct_solvers_agree_and_pcg_converges(shifted):
    st = oracle.assemble(shifted)
    p_ch = oracle.solve_direct(st.H, st.G, method="cholesky")
    p_lu = oracle.solve_direct(st.H, st.G, method="splu")
    for p in (p_ch, p_lu):
        r = st.H @ p.ravel() + st.G.ravel()
        assert np.linalg.norm(r) <= 1e-13 * np.linalg.norm(st.G)
    assert oracle.energy_norm_rel(st.H, p_lu, p_ch) <= 1e-12
    errs = []
    for tol in (1e-4, 1e-8, 1e-12):
        p, it = oracle.block_jacobi_pcg(st.H, st.G, tol)
        r = st.H @ p.ravel() + st.G.ravel()
        assert np.linalg.norm(r) <= tol * np.linalg.norm(st.G)
        errs.append(oracle.energy_norm_rel(st.H, p, p_ch))
    assert errs[0] > errs[1] > errs[2] and errs[2] <= 1e-9


def test_reference_solve_pcg_branch_matches_direct():
    sc = scenes.tiny(n=8, n_pt=200, n_ee=200, lateral=(0.3, 0.6))
    st = oracle.assemble(sc)
    p_d = oracle.solve_direct(st.H, st.G, method="splu")
    p_r = oracle.solve_reference(st.H, st.G, direct_max_dof=0)
    assert oracle.energy_norm_rel(st.H, p_r, p_d) <= 1e-9


# --------------------------------------------------------------------------
# Pins of the contact terms' Hessian weight and of the offset in c_i
# (Section 4.2: the linearized constraint c_i(x_hat) = d_i(x) + grad d_i(x)^T
# (x_hat - x) - delta, and the Newton step's Hessian term mu gamma_i grad d_i
# grad d_i^T, kept for every constraint).

def _two_tets(pt, ee, lam, gamma, kappa=1e4, delta=1e-3, x_hat=None):
    """Tet A with its vertex 0 at p = (0.2, 0.3, 0.05) above the triangle
    (0,0,0), (1,0,0), (0,1,0) of tet B in the plane z = 0 (both positively
    oriented), no fixed nodes."""
    p = np.array([0.2, 0.3, 0.05])
    rest = np.array([p, p + [1, 0, 0], p + [0, 1, 0], p + [0, 0, 1],
                     [0, 0, 0], [0, 1, 0], [1, 0, 0], [0, 0, -1]], dtype=np.float64)
    tets = np.array([[0, 1, 2, 3], [4, 5, 6, 7]], dtype=np.int32)
    n_c = len(pt) + len(ee)
    return dict(name="two_tets", seed=0, rest=rest, tets=tets, E=np.full(2, 1e5), nu=np.full(2, 0.4),
                rho=np.full(2, 1000.0), fixed=np.zeros(8, np.uint8), x=rest.copy(),
                x_hat=rest.copy() if x_hat is None else x_hat, x_tilde=rest.copy(), dt=0.01,
                pt=np.asarray(pt, np.int32).reshape(-1, 4), ee=np.asarray(ee, np.int32).reshape(-1, 4),
                lam=np.full(n_c, float(lam)), gamma=np.full(n_c, float(gamma)), kappa=kappa, delta=delta, tol=1e-8)


def _contact_part(sc):
    """(G, H) of the constraints alone: the scene assembled with and without them."""
    with_c = oracle.assemble(sc)
    bare = dict(sc, pt=np.zeros((0, 4), np.int32), ee=np.zeros((0, 4), np.int32), lam=np.zeros(0),
                gamma=np.zeros(0))
    without = oracle.assemble(bare)
    return with_c, with_c.G - without.G, (with_c.H - without.H).toarray()


# Hand cases.  PT (p, t0, t1, t2) = (0, 4, 6, 5): the closest point of the
# triangle (0,0,0), (1,0,0), (0,1,0) to p = (0.2, 0.3, 0.05) is (0.2, 0.3, 0),
# barycentric (0.5, 0.2, 0.3), so d = 0.05, n = (0, 0, 1), w = (1, -0.5, -0.2, -0.3).
# EE (a0, a1, b0, b1) = (0, 2, 6, 5): edge a runs from p along +y, edge b from
# (1,0,0) to (0,1,0); the closest points are s = 0.5 on a, t = 0.8 on b, so
# d = 0.05, n = (0, 0, 1), w = (1 - s, s, -(1 - t), -t) = (0.5, 0.5, -0.2, -0.8).
HAND = {"pt": ((0, 4, 6, 5), (1.0, -0.5, -0.2, -0.3)),
        "ee": ((0, 2, 6, 5), (0.5, 0.5, -0.2, -0.8))}


@pytest.mark.parametrize("kind", ["pt", "ee"])
def test_contact_blocks_and_gradient_on_hand_case(kind):
    ids, w = HAND[kind]
    w = np.array(w)
    n = np.array([0.0, 0.0, 1.0])
    kappa, gamma, lam = 1e4, 0.6, 1000.0
    rows = [ids]
    sc = _two_tets(rows if kind == "pt" else [], rows if kind == "ee" else [], lam, gamma, kappa)
    st, Gc, Hc = _contact_part(sc)
    assert np.isclose(st.d[0], 0.05, rtol=1e-14) and np.allclose(st.nrm[0], n, atol=1e-14)
    assert np.allclose(st.w[0], w, atol=1e-14)
    # c at x_hat = x is d - delta; g = gamma min(kappa c - lambda, 0) = 0.6 (490 - 1000)
    assert np.isclose(st.c[0], 0.05 - 1e-3, rtol=1e-13)
    gval = gamma * (kappa * (0.05 - 1e-3) - lam)
    assert np.isclose(gval, -306.0)
    for a, v in enumerate(ids):
        assert np.allclose(Gc[v], gval * w[a] * n, rtol=1e-12, atol=1e-9)
    for a, va in enumerate(ids):
        for b, vb in enumerate(ids):
            blk = Hc[3 * va:3 * va + 3, 3 * vb:3 * vb + 3]
            assert np.allclose(blk, kappa * gamma * w[a] * w[b] * np.outer(n, n), rtol=1e-12, atol=1e-6)
    others = np.setdiff1d(np.arange(8), ids)
    assert np.all(Gc[others] == 0.0)
    dofs = (3 * others[:, None] + np.arange(3)).ravel()
    assert np.abs(Hc[dofs]).max() <= 1e-6 and np.abs(Hc[:, dofs]).max() <= 1e-6


@pytest.mark.parametrize("kind", ["pt", "ee"])
def test_constraint_value_offset_and_linearization(kind):
    """c(x_hat) = d - delta + sum_a w_a n . (x_hat_a - x_a), by hand: p moves
    down 0.02 and the constraint's third vertex moves (0.1, 0, 0.01)."""
    ids, w = HAND[kind]
    delta = 2.5e-3
    rows = [ids]
    xh = _two_tets([], [], 0.0, 1.0)["rest"].copy()
    xh[ids[0]] += [0.0, 0.0, -0.02]
    xh[ids[2]] += [0.1, 0.0, 0.01]
    sc = _two_tets(rows if kind == "pt" else [], rows if kind == "ee" else [], 0.0, 1.0, delta=delta, x_hat=xh)
    st = oracle.assemble(sc)
    want = 0.05 - delta + w[0] * (-0.02) + w[2] * 0.01
    assert np.isclose(st.c[0], want, rtol=1e-13)
    sc0 = _two_tets(rows if kind == "pt" else [], rows if kind == "ee" else [], 0.0, 1.0, delta=delta)
    assert np.isclose(oracle.assemble(sc0).c[0], 0.05 - delta, rtol=1e-14)


def test_hessian_is_jacobian_of_gradient_where_nothing_is_projected():
    """All constraints in the branch mu c < lambda (so G's contact part is
    gamma (mu c - lambda) grad d, linear in x_hat) and every tet's 9x9
    Hessian positive definite (so the projection changes nothing): then H is
    exactly the Jacobian of G, and (G(x+eps v) - G(x-eps v)) / 2 eps = H v.
    gamma varies per constraint (not 1), so a dropped or misplaced weight in
    the Hessian fails here even where G is right."""
    sc = free(scenes.tiny(lateral=(0.37, 0.21)))
    rng = np.random.default_rng(17)
    # each cube dilated 5 % about its own centre (twist modes stay positive), small noise
    xh = sc["rest"].copy()
    half = len(xh) // 2
    for sl in (slice(0, half), slice(half, None)):
        cen = xh[sl].mean(axis=0)
        xh[sl] = cen + 1.05 * (xh[sl] - cen)
    xh += rng.normal(0.0, 1e-3, size=xh.shape)
    sc["x_hat"] = xh
    n_c = len(sc["lam"])
    sc["lam"] = np.full(n_c, 2000.0)
    sc["gamma"] = rng.uniform(0.3, 1.7, size=n_c)
    st = oracle.assemble(sc)
    assert np.all(sc["kappa"] * st.c < sc["lam"] - 100.0)           # active branch, with margin
    F = oracle.deformation_gradient(xh, st.tets, st.Dminv)
    ev = np.linalg.eigvalsh(oracle.nh_hessian9(F, st.mu_l, st.lam_l))
    assert ev.min() > 1e-3 * ev.max()                               # nothing to project
    H = st.H.tocsr()
    eps = 1e-6
    for _ in range(3):
        v = rng.normal(size=xh.shape)
        Gp = oracle.assemble(dict(sc, x_hat=xh + eps * v)).G
        Gm = oracle.assemble(dict(sc, x_hat=xh - eps * v)).G
        fd = ((Gp - Gm) / (2 * eps)).ravel()
        Hv = H @ v.ravel()
        assert np.linalg.norm(fd - Hv) <= 1e-6 * np.linalg.norm(Hv)
        # the contact part alone is resolved too (it is a large share of H v here)
        bare = dict(sc, pt=sc["pt"][:0], ee=sc["ee"][:0], lam=sc["lam"][:0], gamma=sc["gamma"][:0])
        Hc_v = Hv - oracle.assemble(bare).H @ v.ravel()
        assert np.linalg.norm(Hc_v) > 1e-3 * np.linalg.norm(Hv)
