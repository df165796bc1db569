#!/usr/bin/env python3
"""Newton-step benchmark on one MI355X: assemble + block-Jacobi PCG to 1e-5.

Workload (default "large"): five 50x50x30-cell Kuhn blocks (2.25M tets,
403,155 nodes, 1.21M DoF) compressed 40 % between fixed planes, 600k
point-triangle + 400k edge-edge constraints, kappa = 1e5; synthetic, seeded.

One "step" is one bf_newton_step call with the state already in HBM:
constraint linearization, merged BSR pattern, elastic/contact assembly (FP64),
preconditioner and FP32 sliced storage, PCG to a relative residual of 1e-5
(FP32 vectors, FP64 reductions and solution), FP64 stats.  `dtype` names the
PCG's arithmetic, where the step spends its time.  Prints one JSON line (see
the fields below); progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json

import numpy as np
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def spmv_bytes(N, nnzb):
    """Algorithmic bytes of one launch of the symmetric SpMV (the roofline's
    unit of work): every stored upper block once, 36 B of FP32 values and a
    4 B column index; a row pointer per row (4(N + 1) B); the vector read and
    the product written (24 B/node).  nnzb counts the stored upper blocks with
    the diagonal."""
    return 40 * nnzb + 4 * (N + 1) + 24 * N


def spmv_design_bytes(N, nnzb):
    """What this design's SpMV must move at least: the n_off = nnzb - N
    off-diagonal upper blocks once (36 B values + 4 B column; the diagonal
    blocks of the scaled matrix are identities and are not stored), one 8 B
    lower reference per block, two slice offsets per row, p and r read (r for
    r^T q) and q written (36 B/node).  The lower half's second read of each
    block is not counted (the same data)."""
    n_off = nnzb - N
    return 48 * n_off + 8 * (N + 1) + 36 * N


def pcg_iteration_bytes(N, nnzb, check_every=1, x_batch=8):
    """The SpMV's design bytes + the update kernel: p, q and r read (36 B/node),
    r and the next p written (24 B/node); every x_batch-th iteration also
    applies the pending x += alpha_j p_j, reading the other x_batch - 1
    directions (12 B/node each) and the FP64 x, and writing x (48 B/node),
    spread over the x_batch iterations; and the factor L (24 B/node) on the
    iterations that test |L r|."""
    return spmv_design_bytes(N, nnzb) + (60 + (48 + 12.0 * (x_batch - 1)) / x_batch + 24.0 / check_every) * N


def copy_ceiling():
    """Device-to-device copy of 512 MiB (read + write bytes per second), the
    bandwidth a plain stream reaches on this device."""
    import torch
    n = 128 * 1024 * 1024
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return {"bytes_read": 4 * n, "bytes_written": 4 * n, "ms": round(ms, 4),
            "gbs_read_plus_write": round(8 * n / (ms * 1e-3) / 1e9, 1)}


COUNTER_FILE = os.path.join(ROOT, "profiles", "k_spmv_large_hbm_counters.md")
# the SpMV and update kernels, and the host rule that plans which slices each SpMV wavefront takes
KERNEL_SOURCES = ["pcg.hip", "assemble.hip", "common.h", "host_rules.cpp"]


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2512_12151_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counter_traffic():
    """HBM bytes per k_spmv launch from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by a plain copy's readings), or
    None when the SpMV sources changed since the counters were taken."""
    import re
    try:
        txt = open(COUNTER_FILE).read()
    except OSError:
        return None
    m_sha = re.search(r"^kernel_sources_sha256: ([0-9a-f]+)", txt, re.M)
    m_tr = re.search(r"^traffic_bytes_per_launch: (\d+)", txt, re.M)
    if not (m_sha and m_tr) or m_sha.group(1) != kernel_sources_sha256():
        return None
    return int(m_tr.group(1))


ASSEMBLY_FILE = os.path.join(ROOT, "profiles", "assembly_large_counters.md")
ASSEMBLY_SOURCES = ["elastic.hip", "assemble.hip", "common.h"]


def assembly_counters():
    """The element and row-assembly kernels' HBM and VALU figures from the
    committed counter summary (JSON on its `assembly_kernels:` line), or None
    when their sources changed since the counters were taken."""
    import hashlib
    import re
    try:
        txt = open(ASSEMBLY_FILE).read()
    except OSError:
        return None
    h = hashlib.sha256()
    for f in ASSEMBLY_SOURCES:
        with open(os.path.join(ROOT, "paper_2512_12151_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    m_sha = re.search(r"^kernel_sources_sha256: ([0-9a-f]+)", txt, re.M)
    m_js = re.search(r"^assembly_kernels: (\{.*\})$", txt, re.M)
    if not (m_sha and m_js) or m_sha.group(1) != h.hexdigest():
        return None
    return json.loads(m_js.group(1))


def cpu_baseline(sc, gpu_iters, frac):
    """The FP64 oracle on a bounded sample of the workload, one thread.

    Sample: the first `frac` of the tets and of each constraint type.  The
    oracle assembles G and H for the sample (linearization, elasticity with
    its numeric projection, inertia, AL terms, DBC) and times FP64
    block-Jacobi PCG iterations on the sample's H; both are scaled by 1/frac
    and the PCG time by the GPU's iteration count to give ms per Newton step
    of the full workload."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import oracle
    sub = dict(sc)
    T = len(sc["tets"])
    sub["tets"] = sc["tets"][: int(frac * T)]
    for k in ("E", "nu", "rho"):
        sub[k] = sc[k][: int(frac * T)]
    npt, nee = int(frac * len(sc["pt"])), int(frac * len(sc["ee"]))
    sub["pt"], sub["ee"] = sc["pt"][:npt], sc["ee"][:nee]
    lam = np.concatenate([sc["lam"][:npt], sc["lam"][len(sc["pt"]):len(sc["pt"]) + nee]])
    sub["lam"], sub["gamma"] = lam, np.ones(len(lam))
    with threadpool_limits(1):
        # per-mesh data of the full mesh (lumped mass over every tet), per-tet
        # arrays restricted to the sample; not timed (per-mesh setup)
        full = oracle.prepare(sc)
        m = len(sub["tets"])
        full.tets, full.Dminv, full.vol, full.A = full.tets[:m], full.Dminv[:m], full.vol[:m], full.A[:m]
        full.mu_l, full.lam_l, full.mat = full.mu_l[:m], full.lam_l[:m], full.mat[:m]
        t0 = time.perf_counter()
        st = oracle.assemble(sub, full)
        t_asm = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.block_jacobi_pcg(st.H, st.G, 0.0, max_iter=4)
        t_a = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.block_jacobi_pcg(st.H, st.G, 0.0, max_iter=24)
        t_b = time.perf_counter() - t0
    t_it = max(t_b - t_a, 0.0) / 20.0
    # the FP64 oracle PCG's own iteration count at this tolerance on this
    # workload, recorded with its reference solution; else the GPU's
    iters, src = gpu_iters, "the GPU's iteration count"
    try:
        import scenes
        with open(os.path.join(ROOT, "tests", "golden", "large_p_ref.json")) as f:
            meta = json.load(f)
        if sc.get("name") == "large" and meta["digest"] == scenes.digest(sc):
            iters = int(meta["fp64_pcg_at_step_tol"]["iterations"])
            src = "the FP64 oracle PCG's own iteration count to 1e-5 on the full workload"
    except (OSError, KeyError, ValueError):
        pass
    ms = (t_asm + t_it * iters) / frac * 1e3
    return {"value": round(ms, 1), "unit": "ms", "cores": 1, "kind": "oracle",
            "sample": (f"first {frac:.0%} of tets and constraints ({len(sub['tets'])} tets, {npt}+{nee} PT+EE): "
                       f"oracle assembly {t_asm:.2f} s and FP64 block-Jacobi PCG {t_it * 1e3:.1f} ms/iteration "
                       f"(one thread), each scaled by 1/{frac:g}; PCG x {iters} iterations ({src})")}


def serve_trace(server, reqs, arrivals, timeout=600.0):
    """Submit reqs[i] at arrivals[i] seconds after the start (a Poisson trace,
    or all at 0 for a capacity run) and poll completions.  Returns per-request
    latency (done - submit, s), the span from the first submit to the last
    completion, statuses, and the mean setup and PCG times (ms)."""
    n = len(reqs)
    lat = np.zeros(n)
    status = np.zeros(n, dtype=int)
    setup, pcg = np.zeros(n), np.zeros(n)
    first, last = None, 0.0
    done = 0
    k = 0
    t0 = time.perf_counter()
    while done < n:
        now = time.perf_counter() - t0
        while k < n and arrivals[k] <= now:
            server.submit(k, reqs[k])
            k += 1
        for i in server.poll():
            _, st, times, rs = server.result(i)
            lat[i] = times["t_done"] - times["t_submit"]
            status[i] = rs
            setup[i], pcg[i] = st["ms_assemble"], st["ms_pcg"]
            first = times["t_submit"] if first is None else min(first, times["t_submit"])
            last = max(last, times["t_done"])
            done += 1
        if now > timeout:
            raise RuntimeError("serving trace did not finish")
        nxt = arrivals[k] - (time.perf_counter() - t0) if k < n else 2e-4
        time.sleep(min(max(nxt, 0.0), 2e-4))
    return lat, last - first, status, float(setup.mean()), float(pcg.mean())


def run_abi_end_to_end(ctx, sc, opts):
    """The same Newton step through the C-ABI with host buffers: a problem
    created from host arrays (per-mesh setup, timed separately), then
    bf_set_state and bf_set_constraints from host memory, bf_newton_step into
    a host array; wall time of the three calls (PCIe copies included).  Median
    of three after one warm-up call."""
    from paper_2512_12151_amd import bfal
    t0 = time.perf_counter()
    pb = bfal.Problem(ctx, sc["tets"], sc["rest"], sc["E"], sc["nu"], sc["rho"], sc["fixed"])
    ms_create = (time.perf_counter() - t0) * 1e3
    ms = []
    for rep in range(4):
        t0 = time.perf_counter()
        pb.set_state(sc["x"], sc["x_hat"], sc["x_tilde"], sc["dt"])
        pb.set_constraints(sc["pt"], sc["ee"], sc["lam"], sc["gamma"], sc["kappa"], sc["delta"])
        _, st, _ = pb.newton_step(**opts)
        if rep:
            ms.append((time.perf_counter() - t0) * 1e3)
    pb.close()
    return {"ms_problem_create": round(ms_create, 2), "ms_state_constraints_step": round(float(np.median(ms)), 2),
            "pcg_iters": st["pcg_iters"],
            "note": "host buffers in and out: x, x_hat, x_tilde, the constraint rows, lambda, gamma copied in, "
                    "p copied out; not the metric (the metric's inputs are already in HBM)"}


def run_bf16(args):
    """The precision variant on the medium workload (120k tets): BF16 copies of
    the scaled blocks inside the FP32/FP64 refinement to a 1e-6 relative
    residual (inner tolerance 0.3), beside plain FP32 PCG to the same 1e-6.
    Per sweep: the FP64 relative residual of the FP32-stored system."""
    import torch

    import scenes
    from paper_2512_12151_amd import bfal
    sc = scenes.make_scene("medium")
    ctx = bfal.Context(0)
    pb = bfal.Problem.from_scene(ctx, sc)
    out = {}
    for name, kw in (("bf16_refine", dict(tol=0.3, refine_tol=1e-6, precision=bfal.BF_PREC_BF16_REFINE)),
                     ("fp32", dict(tol=1e-6))):
        pb.newton_step(max_iter=50000, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st, status = pb.newton_step(max_iter=50000, **kw)
        ms = (time.perf_counter() - t0) * 1e3
        out[name] = {"ms_step": round(ms, 3), "status": status, "pcg_iters": st["pcg_iters"],
                     "sweeps": st["refine_sweeps"], "rel_residual": st["rel_residual"],
                     "ms_pcg": round(st["ms_pcg"], 3)}
        if name == "bf16_refine":
            out[name]["sweep_rel_residual"] = [float("%.3e" % v) for v in st["sweep_rel_residual"]]
    pb.close()
    ctx.close()
    out["workload"] = "medium: 120000 tets, 26620 nodes, 12000 PT + 8000 EE, kappa 1e4, refinement to 1e-6"
    return out


def run_subproblem(args):
    """The rest of Algorithm 2 on the medium workload: Newton steps with the
    FP64 halving line search until a full step (r = 1/2, 1/2, 1 here), then
    the multiplier update.  The large workload's multipliers are drawn apart
    from its state, so its first steps ask for metre-sized moves that the line
    search cuts to r ~ 1/64; it takes tens of Newton steps and is not a bench
    line.  Timed once, after a warm-up call on a fresh problem."""
    import torch

    import scenes
    from paper_2512_12151_amd import bfal
    sc = scenes.make_scene("medium")
    ctx = bfal.Context(0)
    out = {}
    for rep in range(2):
        pb = bfal.Problem.from_scene(ctx, sc)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, _, sst, status = pb.solve_subproblem(tol=args.tol, max_iter=args.max_iter, max_newton=20)
        ms = (time.perf_counter() - t0) * 1e3
        pb.close()
        out = {"workload": "medium", "ms": round(ms, 2), "status": status,
               **{k: (round(v, 6) if isinstance(v, float) else v) for k, v in sst.items()}}
    ctx.close()
    return out


def run_ccd(reps=5):
    """The collision queries of Algorithms 1 and 3 on the large workload with
    its blocks pushed 1 mm per layer into each other (target state on the
    device): MaxStepSize and UpdateActiveSet (from the workload's own active
    set, restored before every call), median of reps calls after one warm-up
    call (which also extracts the surface, once per problem)."""
    import torch

    import scenes
    from paper_2512_12151_amd import bfal
    sc = scenes.make_scene("large")
    xh = torch.from_numpy(scenes.ccd_target(sc, "layers")).to("cuda:0")
    ctx = bfal.Context(0)
    pb = bfal.Problem.from_scene(ctx, sc)
    pb.max_step_size(xh)
    ms_step, ms_upd, st_step, st_upd = [], [], None, None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        alpha, st_step = pb.max_step_size(xh)
        ms_step.append((time.perf_counter() - t0) * 1e3)
    for _ in range(reps):
        pb.set_constraints(sc["pt"], sc["ee"], sc["lam"], sc["gamma"], sc["kappa"], sc["delta"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st_upd = pb.update_active_set(xh)
        ms_upd.append((time.perf_counter() - t0) * 1e3)
    pb.close()
    ctx.close()
    r = lambda v: round(float(v), 3)
    return {"workload": "large, blocks pushed 1 mm per layer (0.4 mm interpenetration per interface)",
            "surface": {"triangles": 110000, "edges": 165000, "vertices": 55010},
            "max_step_size_ms": r(np.median(ms_step)), "alpha": alpha,
            "update_active_set_ms": r(np.median(ms_upd)),
            "device_ms": {"bvh_build": r(st_step["ms_tree"]), "query_accd": r(st_step["ms_query"]),
                          "set_rebuild": r(st_upd["ms_update"])},
            "candidates": [st_step["candidates_pt"], st_step["candidates_ee"]],
            "colliding": [st_step["colliding_pt"], st_step["colliding_ee"]],
            "added": [st_upd["added_pt"], st_upd["added_ee"]], "removed": st_upd["removed"],
            "active_after": [st_upd["n_pt"], st_upd["n_ee"]]}


def run_variants(ctx, t, sc, opts, base):
    """The other materials and friction (Table 2, Appendix A) on the large
    workload: one Newton step each (after a warm-up step) with every tet stable
    Neo-Hookean or corotated linear, and with Neo-Hookean plus the friction set
    captured from the workload's 1M contacts (eps_v = 1e-3 as in Table 2;
    mu_f = 1e-5 because the workload's multipliers, up to 1e4, are drawn far
    above what a step on its 1e-2 kg nodes produces: mu_f keeps the sticking
    stiffness 2 mu_f lambda / (eps_v h) below kappa, which the FP32 blocks can
    hold).  The assembly phase holds the element kernel of the material and
    the friction terms; the PCG solves a different matrix in each, so its
    iteration count is reported beside the time."""
    import torch

    from paper_2512_12151_amd import bfal
    T = len(sc["tets"])
    out = {}
    keys = ("ms_lin", "ms_pattern", "ms_assemble", "ms_pcg")

    def step(pb):
        res = torch.empty((len(sc["rest"]), 3), dtype=torch.float64, device="cuda:0")
        pb.newton_step(out=res, **opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st, status = pb.newton_step(out=res, **opts)
        ms = (time.perf_counter() - t0) * 1e3
        return {"ms_step": round(ms, 3), "status": status, "pcg_iters": st["pcg_iters"],
                **{k: round(st[k], 3) for k in keys}}

    for name, code in (("snh", 1), ("cor", 2)):
        mat = torch.full((T,), code, dtype=torch.int32, device="cuda:0")
        pb = bfal.Problem(ctx, t["tets"], t["rest"], t["E"], t["nu"], t["rho"], t["fixed"], material=mat)
        pb.set_state(t["x"], t["x_hat"], t["x_tilde"], sc["dt"])
        pb.set_constraints(t["pt"], t["ee"], t["lam"], t["gamma"], sc["kappa"], sc["delta"])
        out[name] = step(pb)
        pb.close()
        log(f"material {name}: {out[name]}")
    base.set_friction(1e-5, 1e-3)
    out["nh_friction"] = step(base)
    base.set_friction(0.0)
    log(f"friction: {out['nh_friction']}")
    return out


def run_time_step(reps=3):
    """Algorithm 1 with friction: two stacked 8^3-cell cubes (12,288 tets), the
    upper one thrown down at 0.5 m/s and sideways at 0.2 m/s onto the lower one;
    the first step lands it (contacts appear), the second, timed, carries the
    active set and multipliers and captures the friction set from them
    (mu_f = 0.5, eps_v = 1e-3, K_min = 6 as the paper uses with friction).
    Median of reps runs of the second step on fresh problems."""
    import scenes
    from paper_2512_12151_amd import bfal
    sc = dict(scenes.falling_cubes(n=8, jitter=1e-5))
    N, h = len(sc["x"]), sc["dt"]
    sc["x_tilde"] = sc["x_tilde"].copy()
    sc["x_tilde"][N // 2:, 0] += h * 0.2
    ctx = bfal.Context(0)
    kw = dict(tol=1e-5, mu_f=0.5, eps_v=1e-3, k_min=6)
    ms, last = [], None
    for _ in range(reps):
        pb = bfal.Problem.from_scene(ctx, sc)
        x1, v1, st1, _ = pb.time_step(**kw)
        pb.set_state(x1, x1.copy(), x1 + h * v1, h)
        t0 = time.perf_counter()
        _, _, last, status = pb.time_step(**kw)
        ms.append((time.perf_counter() - t0) * 1e3)
        pb.close()
    ctx.close()
    r = lambda v: round(float(v), 3)
    return {"workload": "two 8^3-cell cubes (12288 tets), thrown at (0.2, 0, -0.5) m/s, the step after landing",
            "ms_step": r(np.median(ms)), "status": status, "outer_iters": last["outer_iters"],
            "newton_iters": last["newton_iters"], "pcg_iters": last["pcg_iters"],
            "ms_subproblem": r(last["ms_subproblem"]), "ms_ccd": r(last["ms_ccd"]),
            "active_after": [last["n_pt"], last["n_ee"]]}


def run_serve(n_req, seed=5, loads=(0.8, 1.2, 2.0)):
    """Serving (continuous batching) on a stream of two-stacked-cube requests
    (tets ~ LogU[2k, 300k]).  The one-at-a-time service time is measured first
    (64 requests back to back on the same engine with one slot); Poisson traces
    at `loads` x that service rate are then served by the batching server and
    one at a time; a capacity run submits everything at once; a forced small
    budget (1.25 x the largest request's footprint) repeats the first trace."""
    import torch

    import scenes
    from paper_2512_12151_amd import bfal
    log(f"serve: generating {n_req} requests")
    reqs = [scenes.serve_request(i) for i in range(n_req)]
    free, _ = torch.cuda.mem_get_info()
    budget = int(0.9 * free)

    def summary(lat, span, status, su, pc):
        return {"p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
                "mean_ms": round(float(lat.mean()) * 1e3, 3),
                "steps_per_s": round(len(lat) / span, 2), "errors": int((status < 0).sum()),
                "mean_setup_ms": round(su, 3), "mean_pcg_ms": round(pc, 3)}

    def serve(reqs_, arrivals, max_active, budget_=budget):
        sv = bfal.Server(0, hbm_budget=budget_, max_active=max_active, iters_per_round=8)
        try:
            return summary(*serve_trace(sv, reqs_, arrivals))
        finally:
            sv.close()

    cal = min(64, n_req)
    one = serve(reqs[:cal], np.zeros(cal), 1)
    service = 1.0 / one["steps_per_s"]
    out = {"requests": n_req, "one_at_a_time_service_ms": round(service * 1e3, 3), "hbm_budget_bytes": budget,
           "capacity": {"one_at_a_time": one, "batched": serve(reqs, np.zeros(n_req), 64)}}
    log(f"serve capacity: {out['capacity']}")
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0, size=n_req)
    for load in loads:
        rate = load / service
        arrivals = np.cumsum(gaps / rate)
        arrivals -= arrivals[0]
        key = f"load_{load:g}"
        out[key] = {"arrival_rate_per_s": round(rate, 2), "batched": serve(reqs, arrivals, 64),
                    "one_at_a_time": serve(reqs, arrivals, 1)}
        log(f"serve {key}: {out[key]}")
    small = int(1.25 * max(bfal.footprint_bytes(len(r["rest"]), len(r["tets"]), len(r["pt"]) + len(r["ee"]))
                           for r in reqs))
    rate = loads[0] / service
    arrivals = np.cumsum(gaps / rate)
    arrivals -= arrivals[0]
    out["small_budget"] = {"hbm_budget_bytes": small, "load": loads[0], "batched": serve(reqs, arrivals, 64, small)}
    log(f"serve small budget: {out['small_budget']}")
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="large", choices=["large", "medium", "tiny"])
    ap.add_argument("--tol", type=float, default=1e-5)
    ap.add_argument("--check-every", type=int, default=4,
                    help="PCG iterations between tests of the unscaled residual |L r| against tol")
    ap.add_argument("--cpu-sample", type=float, default=0.1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--max-iter", type=int, default=200000,
                    help="PCG iteration cap (lower it only for counter-collection runs)")
    ap.add_argument("--no-subproblem", dest="subproblem", action="store_false",
                    help="skip the SolveSubproblem measurement (Newton loop with line search, multiplier update)")
    ap.add_argument("--no-variants", dest="variants", action="store_false",
                    help="skip the material / friction step variants and the time-step leg")
    ap.add_argument("--no-ccd", dest="ccd", action="store_false",
                    help="skip the collision-query measurement (MaxStepSize, UpdateActiveSet)")
    ap.add_argument("--no-bf16", dest="bf16", action="store_false",
                    help="skip the BF16-blocks-with-refinement leg on the medium workload")
    ap.add_argument("--serve-requests", type=int, default=512,
                    help="requests of the serving trace (0 skips the serving measurement)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="time a plain device-to-device copy of 512 MiB (bandwidth ceiling and the reference "
                         "for scaling HBM counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU design is described in "
              "DESIGN.md and not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import scenes
    from paper_2512_12151_amd import bfal

    if args.copy_probe:
        print(json.dumps(copy_ceiling()), flush=True)
        return

    log(f"generating workload {args.workload}")
    sc = scenes.make_scene(args.workload)
    N, T = len(sc["rest"]), len(sc["tets"])
    n_c = len(sc["pt"]) + len(sc["ee"])
    dev = torch.device("cuda:0")
    t = {k: torch.from_numpy(np.ascontiguousarray(sc[k])).to(dev)
         for k in ("tets", "rest", "E", "nu", "rho", "fixed", "x", "x_hat", "x_tilde", "pt", "ee", "lam", "gamma")}
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    ctx = bfal.Context(0, stream=stream.cuda_stream)
    log(f"setup: {N} nodes, {T} tets, {n_c} constraints")
    pb = bfal.Problem(ctx, t["tets"], t["rest"], t["E"], t["nu"], t["rho"], t["fixed"])
    pb.set_state(t["x"], t["x_hat"], t["x_tilde"], sc["dt"])
    pb.set_constraints(t["pt"], t["ee"], t["lam"], t["gamma"], sc["kappa"], sc["delta"])
    out = torch.empty((N, 3), dtype=torch.float64, device=dev)
    opts = dict(tol=args.tol, max_iter=args.max_iter, poll_every=64, check_every=args.check_every)
    for w in range(args.warmup):
        _, st, status = pb.newton_step(out=out, **opts)
        log(f"warmup {w}: status {status}, {st['pcg_iters']} PCG iterations, rel residual {st['rel_residual']:.2e}")
    # every step bracketed by events on the library's stream (torch's current
    # stream, handed to the context); the wall clock spans all of them
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = []
    last = None
    for k in range(args.steps):
        ev[k][0].record(stream)
        _, last, status = pb.newton_step(out=out, **opts)
        ev[k][1].record(stream)
        iters.append(last["pcg_iters"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_step = elapsed / args.steps * 1e3
    ms_events = [a.elapsed_time(b) for a, b in ev]
    log(f"timed {args.steps} steps: {ms_step:.2f} ms/step, event median {np.median(ms_events):.2f}, "
        f"iterations {iters}")
    # dominant kernel: time the SpMV launches of one more step with HIP events on the library's stream
    _, tst, _ = pb.newton_step(out=out, time_spmv=256, **opts)
    nnzb = int(last["nnzb"])
    sb = spmv_bytes(N, nnzb)
    spmv_ms = tst["ms_spmv_avg"]
    achieved = sb / (spmv_ms * 1e-3) / 1e9
    it_mean = float(np.mean(iters))
    pcg_gbs = pcg_iteration_bytes(N, nnzb, args.check_every) * last["pcg_iters"] / (last["ms_pcg"] * 1e-3) / 1e9
    cc = copy_ceiling()
    line = {
        "metric": "Newton-step assemble+PCG ms @1e-5 rel residual",
        "value": round(ms_step, 3),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {T} tets, {N} nodes, {3 * N} DoF, {len(sc['pt'])} PT + "
                               f"{len(sc['ee'])} EE constraints, kappa {sc['kappa']:g}, PCG tol {args.tol:g} "
                               f"(|L r| tested every {args.check_every} iterations)",
                   "parallelism": "single GPU"},
        "ms_step_events": {"median": round(float(np.median(ms_events)), 3), "min": round(min(ms_events), 3),
                           "max": round(max(ms_events), 3)},
        "pcg_iters": it_mean,
        "pcg_iters_per_s": round(last["pcg_iters"] / (last["ms_pcg"] * 1e-3), 1),
        "phase_ms": {k: round(last[k], 3) for k in ("ms_lin", "ms_pattern", "ms_assemble", "ms_pcg")},
        "pcg_design_gbs": round(pcg_gbs, 1),
        "nnzb": nnzb,
        "rel_residual": last["rel_residual"],
        "roofline": {"bound": "hbm", "kernel": "k_spmv", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": counter_traffic(),
                     "traffic_scope": "bytes past L2 (rocprofv3 FETCH_SIZE and WRITE_SIZE per launch, scaled by a "
                                      "plain copy's readings); Infinity Cache hits are included",
                     "bytes_per_launch": sb, "bytes_formula": "40 nnzb + 4 (N + 1) + 24 N",
                     "design_bytes_per_launch": spmv_design_bytes(N, nnzb),
                     "design_frac": round(spmv_design_bytes(N, nnzb) / (spmv_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "avg_ms": round(spmv_ms, 5), "launches_timed": tst["spmv_timed"],
                     "copy_ceiling_gbs": cc["gbs_read_plus_write"],
                     "frac_of_copy_ceiling": round(achieved / cc["gbs_read_plus_write"], 4)},
    }
    line["assembly_kernels"] = assembly_counters()
    line["abi_end_to_end"] = run_abi_end_to_end(ctx, sc, opts)
    log(f"abi end to end: {line['abi_end_to_end']}")
    if args.subproblem:
        # FP64 energy evaluation (the line search's unit of work) on this workload
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            pb.energy()
        t_energy = (time.perf_counter() - t0) / 5 * 1e3
    if args.variants:
        line["variants"] = run_variants(ctx, t, sc, opts, pb)
    pb.close()
    if args.bf16:
        line["bf16_refine"] = run_bf16(args)
        log(f"bf16: {line['bf16_refine']}")
    if args.subproblem:
        line["subproblem"] = run_subproblem(args)
        line["subproblem"]["energy_eval_ms_" + args.workload] = round(t_energy, 3)
        log(f"subproblem: {line['subproblem']}")
    if args.variants:
        line["time_step"] = run_time_step()
        log(f"time step: {line['time_step']}")
    if args.ccd:
        line["ccd"] = run_ccd()
        log(f"ccd: {line['ccd']}")
    if args.serve_requests > 0:
        line["serve"] = run_serve(args.serve_requests)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a bounded sample)")
        line["cpu_baseline"] = cpu_baseline(sc, int(round(it_mean)), args.cpu_sample)
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
