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
