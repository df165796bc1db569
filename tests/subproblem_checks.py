"""Checks of a GPU SolveSubproblem result (Algorithm 2) that the oracle can
make at any size without its direct solves: the FP64 total energy at the start
and at the returned state, the energy decrease, untouched fixed nodes, the
multiplier/decay update at the returned state and the violation statistic.

Bars: L within 1e-9 relative (both sides FP64); the update bit-for-bit in its
branch (gamma), constraints within 1e-9 of the branch point c_i =
lambda_i / kappa excepted; lambda' = lambda - kappa c within 1e-9 relative plus
kappa * 1e-11: the two sides compute c_i in FP64 by different closest-point
arithmetic, and for edge pairs at the generators' smallest angle (sin^2 = 1e-4)
the 2x2 closest-point system amplifies rounding by up to 1e4, so c_i may differ
by ~1e-12 and lambda' by kappa times that."""
import numpy as np

import oracle
from oracle import subproblem as osp


def check_subproblem(sc, xh, lam, gam, stats, decay=0.9, prep=None):
    prep = oracle.prepare(sc) if prep is None else prep
    L0 = osp.energy(sc, prep, sc["x_hat"])
    L1 = osp.energy(sc, prep, xh)
    assert abs(stats["energy_initial"] - L0) <= 1e-9 * abs(L0)
    assert abs(stats["energy_final"] - L1) <= 1e-9 * abs(L1)
    assert stats["energy_final"] < stats["energy_initial"]
    fixed = sc["fixed"].astype(bool)
    assert np.array_equal(xh[fixed], sc["x_hat"][fixed])
    lam_o, gam_o, act_o = osp.dual_update(sc, xh, Gamma=decay)
    c = osp.constraint_values_at(sc, xh)
    ratio = sc["lam"] / sc["kappa"]
    margin = np.abs(c - ratio) > 1e-9 * np.maximum(1.0, np.abs(ratio))
    dl = np.abs(lam - lam_o)[margin]
    print(f"update: max |dlambda| {dl.max() if dl.size else 0.0:.3e} (kappa {sc['kappa']:.0e})", flush=True)
    assert np.array_equal(gam[margin], gam_o[margin])
    assert np.allclose(lam[margin], lam_o[margin], rtol=1e-9, atol=1e-11 * sc["kappa"])
    assert stats["active"] == int(act_o.sum()) or not margin.all()
    assert abs(stats["max_violation"] - float(np.maximum(0.0, -c).max())) <= 1e-12
    return L0, L1
