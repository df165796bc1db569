"""Continuous-batching server (bf_server_*) through the C-ABI.

Every request's result must be the same alone and in the mix: the batched
kernels give each request its own workgroups, partial sums and scalars, in the
same order as a lone bf_newton_step, so the bar is bitwise equality with the
single-request path (same p, same iteration count).  Each result is also held
to the FP64 oracle at the solve tolerance, and the HBM budget is enforced."""
import time

import numpy as np
import pytest

import oracle
import scenes

pytestmark = pytest.mark.gpu

# small requests of different sizes (two stacked cubes, the serving recipe)
IDS = [3, 7, 11, 19, 23, 31]
_scenes = {}


def scene(i):
    if i not in _scenes:
        _scenes[i] = scenes.serve_request(i)
    return _scenes[i]


@pytest.fixture(scope="module")
def bf():
    from paper_2512_12151_amd import bfal
    return bfal


@pytest.fixture(scope="module")
def alone(bf):
    ctx = bf.Context(0)
    out = {}
    for i in IDS:
        pb = bf.Problem.from_scene(ctx, scene(i))
        p, st, status = pb.newton_step(tol=1e-5, max_iter=20000)
        out[i] = (p, st)
        pb.close()
    ctx.close()
    return out


def run_server(bf, server, ids, stagger=0.0, timeout=120.0):
    for k, i in enumerate(ids):
        server.submit(i, scene(i), tol=1e-5, max_iter=20000)
        if stagger:
            time.sleep(stagger)
    got = {}
    t0 = time.time()
    while len(got) < len(ids):
        for i in server.poll():
            got[i] = server.result(i)
        assert time.time() - t0 < timeout, "server did not finish"
        time.sleep(0.002)
    return got


@pytest.mark.parametrize("max_active,stagger", [(64, 0.0), (3, 0.002), (1, 0.0)])
def test_results_same_alone_and_in_the_mix(bf, alone, max_active, stagger):
    print(f"case max_active={max_active} stagger={stagger}", flush=True)
    sv = bf.Server(0, hbm_budget=4 << 30, max_active=max_active, iters_per_round=8)
    got = run_server(bf, sv, IDS, stagger)
    sv.close()
    for i in IDS:
        p, st, times, status = got[i]
        assert status == bf.BF_OK
        p1, st1 = alone[i]
        assert st["pcg_iters"] == st1["pcg_iters"]
        assert np.array_equal(p, p1), f"request {i} differs from its lone solve"
        assert times["t_submit"] <= times["t_admit"] <= times["t_done"]


def test_results_against_oracle(bf, alone):
    for i in IDS[:3]:
        sc = scene(i)
        st = oracle.assemble(sc)
        p_ref = oracle.solve_reference(st.H, st.G)
        p64, _ = oracle.block_jacobi_pcg(st.H, st.G, 1e-5)
        err = oracle.energy_norm_rel(st.H, alone[i][0], p_ref)
        err64 = oracle.energy_norm_rel(st.H, p64, p_ref)
        print(f"serve request {i}: N={len(sc['rest'])} err={err:.3e} fp64 pcg err={err64:.3e}", flush=True)
        assert err <= 2.0 * err64 + 1e-5


def decile_ids(n_trace=512):
    """One request per size decile of the serving trace: the request at the
    middle of each tenth of the trace sorted by cube size (the size rule of
    the serving recipe, read from its seeded generator)."""
    from scenes import configs
    ns = []
    for i in range(n_trace):
        T = np.exp(configs._rng(1000 + i, "size").uniform(np.log(2e3), np.log(3e5)))
        ns.append(int(np.clip(np.rint(np.cbrt(T / 12.0)), 6, 29)))
    order = np.argsort(np.array(ns), kind="stable")
    return [int(order[int((k + 0.5) / 10 * n_trace)]) for k in range(10)]


@pytest.mark.timeout(900)
def test_every_size_decile_against_oracle(bf):
    """One request per size decile (cubes of 6^3 to 27^3 cells, 2.6k to 236k
    tets) through the batching server in one mix, each held to the FP64
    oracle in the energy norm: no worse than twice the oracle's own FP64 PCG
    at the same tolerance, plus 1e-5."""
    ids = decile_ids()
    sv = bf.Server(0, hbm_budget=16 << 30, max_active=64, iters_per_round=8)
    got = run_server(bf, sv, ids, timeout=300.0)
    sv.close()
    for i in ids:
        sc = scene(i)
        p, st_gpu, _, status = got[i]
        assert status == bf.BF_OK
        st = oracle.assemble(sc)
        p_ref = oracle.solve_reference(st.H, st.G)
        p64, it64 = oracle.block_jacobi_pcg(st.H, st.G, 1e-5)
        err = oracle.energy_norm_rel(st.H, p, p_ref)
        err64 = oracle.energy_norm_rel(st.H, p64, p_ref)
        print(f"decile request {i}: {len(sc['tets'])} tets, {len(sc['pt']) + len(sc['ee'])} constraints, "
              f"iterations {st_gpu['pcg_iters']} (fp64 {it64}), err {err:.3e} (fp64 pcg {err64:.3e})", flush=True)
        assert err <= 2.0 * err64 + 1e-5


def test_materials_in_the_mix(bf):
    """Requests with per-tet material codes (stable Neo-Hookean, corotated
    linear, mixed) are served like Neo-Hookean ones: bitwise the lone step."""
    ids = [3, 7, 11]
    mats = {}
    for k, i in enumerate(ids):
        sc = dict(scene(i))
        T = len(sc["tets"])
        mats[i] = [np.full(T, 1, np.int32), np.full(T, 2, np.int32), np.arange(T, dtype=np.int32) % 3][k]
        sc["material"] = mats[i]
        _scenes[("mat", i)] = sc
    ctx = bf.Context(0)
    lone = {}
    for i in ids:
        pb = bf.Problem.from_scene(ctx, _scenes[("mat", i)])
        lone[i] = pb.newton_step(tol=1e-5, max_iter=20000)[0]
        pb.close()
    ctx.close()
    sv = bf.Server(0, hbm_budget=4 << 30, max_active=8, iters_per_round=8)
    for i in ids:
        sv.submit(i, _scenes[("mat", i)], tol=1e-5, max_iter=20000)
    got = {}
    t0 = time.time()
    while len(got) < len(ids):
        for i in sv.poll():
            got[i] = sv.result(i)
        assert time.time() - t0 < 120.0
        time.sleep(0.002)
    sv.close()
    for i in ids:
        assert got[i][3] == bf.BF_OK
        assert np.array_equal(got[i][0], lone[i])


def test_submit_validates_like_the_single_problem_calls(bf):
    """bf_server_submit applies the host checks at once (bf_check_*): an
    out-of-range constraint index, a non-positive step and a repeated vertex
    come back from the submit call itself."""
    sv = bf.Server(0, hbm_budget=1 << 30, max_active=2)
    sc = dict(scene(3))
    bad = dict(sc)
    pt = sc["pt"].copy()
    pt[0, 2] = len(sc["rest"]) + 5
    bad["pt"] = pt
    with pytest.raises(bf.BfalError) as e:
        sv.submit(1, bad)
    assert e.value.status == -1
    with pytest.raises(bf.BfalError) as e:
        sv.submit(2, dict(sc, dt=0.0))
    assert e.value.status == -1
    pt = sc["pt"].copy()
    pt[1, 1] = pt[1, 0]
    with pytest.raises(bf.BfalError) as e:
        sv.submit(3, dict(sc, pt=pt))
    assert e.value.status == -5
    assert sv.stats()["pending"] == 0
    sv.close()


def test_budget_admission_and_rejection(bf, alone):
    sizes = {i: bf.footprint_bytes(len(scene(i)["rest"]), len(scene(i)["tets"]),
                                   len(scene(i)["pt"]) + len(scene(i)["ee"])) for i in IDS}
    # room for the largest request only: requests run one or two at a time
    budget = max(sizes.values()) + 1
    sv = bf.Server(0, hbm_budget=budget, max_active=64, iters_per_round=4)
    got = run_server(bf, sv, IDS)
    for i in IDS:
        assert got[i][3] == bf.BF_OK
        assert np.array_equal(got[i][0], alone[i][0])
    assert sv.stats()["used_bytes"] == 0
    sv.close()
    # a request larger than the whole budget is rejected with ERR_BUDGET
    small = min(sizes.values())
    sv = bf.Server(0, hbm_budget=small, max_active=4, iters_per_round=4)
    big = max(sizes, key=sizes.get)
    got = run_server(bf, sv, [big])
    assert got[big][3] == -7   # BF_ERR_BUDGET
    sv.close()
