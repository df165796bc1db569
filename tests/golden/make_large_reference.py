"""Writes the reference solution of the large workload's Newton step.

Calls only the FP64 oracle (and the seeded scene generator): the oracle's
assembly of G and H, then its FP64 block-Jacobi PCG (x0 = 0) to a relative
residual of 1e-12, which stands in for the direct solve at 1.21M unknowns.
On the way it records the same PCG's iterate and iteration count where the
residual first meets 1e-5, the tolerance the GPU step is run at: that is the
FP64 solver's own error at that tolerance, reported beside the GPU's.

Outputs (next to this script):
  large_p_ref.npy   p* as float32 [N, 3]
  large_p_ref.json  scene digest, iteration counts, the FP64 PCG's energy-norm
                    error at 1e-5, and the error the float32 storage of p*
                    itself adds.

Run: python tests/golden/make_large_reference.py   (about an hour, one core)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import scenes  # noqa: E402

TOL_STEP = 1e-5
TOL_REF = 1e-12


def main():
    t0 = time.time()
    sc = scenes.make_scene("large")
    dig = scenes.digest(sc)
    st = oracle.assemble(sc)
    print(f"assembled in {time.time() - t0:.0f} s", flush=True)
    rec = {TOL_STEP: None}
    p_ref, it_ref = oracle.block_jacobi_pcg(st.H, st.G, TOL_REF, max_iter=400000, record=rec)
    p_step, it_step = rec[TOL_STEP]
    b = -st.G.ravel()
    res_ref = float(np.linalg.norm(st.H @ p_ref.ravel() - b) / np.linalg.norm(b))
    res_step = float(np.linalg.norm(st.H @ p_step.ravel() - b) / np.linalg.norm(b))
    err_step = oracle.energy_norm_rel(st.H, p_step, p_ref)
    p32 = p_ref.astype(np.float32)
    err_store = oracle.energy_norm_rel(st.H, p32.astype(np.float64), p_ref)
    np.save(os.path.join(HERE, "large_p_ref.npy"), p32)
    meta = {
        "scene": "large", "digest": dig,
        "reference": {"solver": "FP64 block-Jacobi PCG, x0 = 0", "tol": TOL_REF, "iterations": it_ref,
                      "rel_residual": res_ref},
        "fp64_pcg_at_step_tol": {"tol": TOL_STEP, "iterations": it_step, "rel_residual": res_step,
                                 "energy_norm_error": err_step},
        "float32_storage_energy_norm_error": err_store,
        "seconds": time.time() - t0,
    }
    with open(os.path.join(HERE, "large_p_ref.json"), "w") as f:
        json.dump(meta, f, indent=1)
    print(json.dumps(meta, indent=1), flush=True)


if __name__ == "__main__":
    main()
