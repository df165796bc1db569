"""Writes the reference solution of the large workload's Newton step.

Calls only the FP64 oracle (and the seeded scene generator): the oracle's
assembly of G and H, then its FP64 block-Jacobi PCG (x0 = 0) to a relative
residual of 1e-12, which stands in for the direct solve at 1.21M unknowns.
On the way it records the same PCG's iterate and iteration count where the
residual first meets 1e-5, the tolerance the GPU step is run at: that is the
FP64 solver's own error at that tolerance, reported beside the GPU's.

A second stage bounds how far FP32 storage of the matrix alone moves the
solution (the floor any solver on FP32 blocks works above).  It models the
stored system on the oracle's H: the block-Jacobi scaled matrix
H_hat = M H M^T (M = L^{-1}, D_v = L_v L_v^T per 3x3 diagonal block, FP64)
with identity diagonal blocks and its off-diagonal blocks rounded to FP32,
and b_hat = M b rounded to FP32.  Its exact solution differs from
x* = L^T p* by delta = H_hat32^{-1} (b_hat32 - H_hat32 x*), and
|delta|_{H_hat32} approximates |L^{-T} delta|_H.  CG from 0 on that system
gives iterates d_k with f^T d_k rising to f^T H_hat32^{-1} f = |delta|^2,
so the value after a fixed number of iterations is a lower bound.

Outputs (next to this script):
  large_p_ref.npy   p* as float32 [N, 3]
  large_p_ref.json  scene digest, iteration counts, the FP64 PCG's energy-norm
                    error at 1e-5, the error the float32 storage of p* itself
                    adds, and the FP32-storage floor (lower bound, relative to
                    |p*|_H) with its CG iteration count.

Run: python tests/golden/make_large_reference.py   (the reference solve takes
about three hours, the floor about twenty minutes; a stage whose output is
already there is skipped)
"""
import json
import os
import sys
import time

import numpy as np
import scipy.sparse as sp

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import scenes  # noqa: E402

TOL_STEP = 1e-5
TOL_REF = 1e-12
FLOOR_ITERS = 10000
NPY = os.path.join(HERE, "large_p_ref.npy")
JSN = os.path.join(HERE, "large_p_ref.json")


def reference(sc, st, dig, t0):
    rec = {TOL_STEP: None}
    p_ref, it_ref = oracle.block_jacobi_pcg(st.H, st.G, TOL_REF, max_iter=400000, record=rec)
    p_step, it_step = rec[TOL_STEP]
    b = -st.G.ravel()
    res_ref = float(np.linalg.norm(st.H @ p_ref.ravel() - b) / np.linalg.norm(b))
    res_step = float(np.linalg.norm(st.H @ p_step.ravel() - b) / np.linalg.norm(b))
    err_step = oracle.energy_norm_rel(st.H, p_step, p_ref)
    p32 = p_ref.astype(np.float32)
    err_store = oracle.energy_norm_rel(st.H, p32.astype(np.float64), p_ref)
    np.save(NPY, p32)
    return {
        "scene": "large", "digest": dig,
        "reference": {"solver": "FP64 block-Jacobi PCG, x0 = 0", "tol": TOL_REF, "iterations": it_ref,
                      "rel_residual": res_ref},
        "fp64_pcg_at_step_tol": {"tol": TOL_STEP, "iterations": it_step, "rel_residual": res_step,
                                 "energy_norm_error": err_step},
        "float32_storage_energy_norm_error": err_store,
        "seconds": time.time() - t0,
    }


def storage_floor(st, p_ref, iters):
    """Lower bound of the energy-norm distance between p* and the exact solution
    of the FP32-stored scaled system, relative to |p*|_H (see the module text),
    and the CG iterations it took."""
    H = st.H.tocsr()
    n = H.shape[0]
    N = n // 3
    idx = np.arange(N)
    D = np.empty((N, 3, 3))
    for i in range(3):
        for j in range(3):
            D[:, i, j] = np.asarray(H[3 * idx + i, 3 * idx + j]).ravel()
    L = np.linalg.cholesky(D)
    M = np.linalg.inv(L)
    Mb = sp.block_diag(list(M), format="csr")
    Hh = (Mb @ H @ Mb.T).tocsr()
    rows = np.repeat(np.arange(n), np.diff(Hh.indptr))
    off = rows // 3 != Hh.indices // 3
    H32 = sp.csr_matrix((np.where(off, Hh.data.astype(np.float32).astype(np.float64), 0.0), Hh.indices, Hh.indptr),
                        shape=Hh.shape)
    H32.eliminate_zeros()
    H32 = (H32 + sp.identity(n, format="csr")).tocsr()
    b32 = (Mb @ (-st.G.ravel())).astype(np.float32).astype(np.float64)
    xs = np.einsum("nji,nj->ni", L, p_ref.reshape(N, 3)).ravel()   # x* = L^T p*
    f = b32 - H32 @ xs
    nref2 = float(p_ref.ravel() @ (H @ p_ref.ravel()))
    d = np.zeros(n)
    r = f.copy()
    p = r.copy()
    rr = r @ r
    its = iters
    for k in range(iters):
        q = H32 @ p
        pq = p @ q
        if not pq > 0.0:   # the rounded system is not positive definite along p: stop with the bound so far
            its = k
            break
        a = rr / pq
        d += a * p
        r -= a * q
        rr_new = r @ r
        p = r + (rr_new / rr) * p
        rr = rr_new
    return float(np.sqrt(max(f @ d, 0.0) / nref2)), its


def main():
    t0 = time.time()
    sc = scenes.make_scene("large")
    dig = scenes.digest(sc)
    st = oracle.assemble(sc)
    print(f"assembled in {time.time() - t0:.0f} s", flush=True)
    meta = None
    if os.path.exists(NPY) and os.path.exists(JSN):
        with open(JSN) as f:
            meta = json.load(f)
        if meta.get("digest") != dig:
            meta = None
    if meta is None:
        meta = reference(sc, st, dig, t0)
    if "float32_storage_floor" not in meta:
        p_ref = np.load(NPY).astype(np.float64)
        t1 = time.time()
        bound, its = storage_floor(st, p_ref, FLOOR_ITERS)
        meta["float32_storage_floor"] = {
            "energy_norm_lower_bound": bound, "cg_iterations": its,
            "model": "block-Jacobi scaled H (FP64 factors) with off-diagonal blocks and right-hand side rounded "
                     "to FP32, identity diagonal blocks", "seconds": time.time() - t1}
    with open(JSN, "w") as f:
        json.dump(meta, f, indent=1)
    print(json.dumps(meta, indent=1), flush=True)


if __name__ == "__main__":
    main()
