"""Plain FP64 CPU oracle for one time step (Algorithm 1).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Algorithm 1 (Section 4.1): starting from x^[0] = x_hat^[0] = x^t (moving
boundary nodes of x_hat^[0] already at their targets, Section 5.3), repeat
  x_hat^[k+1] = SolveSubproblem(x_tilde, x^[k], x_hat^[k], C^[k])   (Algorithm 2)
  C^[k+1]     = UpdateActiveSet(x^[k], x_hat^[k], C^[k])            (Algorithm 3)
  alpha       = MaxStepSize(x^[k], x_hat^[k+1])
  x^[k+1]     = (1 - alpha) x^[k] + alpha x_hat^[k+1]
  beta        = (1 - alpha) beta once k + 1 >= K_min
while beta > eps; the step returns x^[k] and v = (x^[k] - x^t) / h.  Section 6
uses eps = 1e-3 and K_min = 2.  Section 5.2: the penalty may start at
mu_init = C max_i (grad^2 E)_ii, and mu doubles (delta halves) when alpha
stays below 1e-4 for 50 consecutive iterations.

Readings (listed in the design doc):
  * UpdateActiveSet runs on the subproblem's *input* x_hat^[k], as the
    algorithm writes it: x^[k] lies on the last CCD path, so x^[k] -> x_hat^[k]
    is the remainder of that path, where the pairs that blocked it are; it
    sees the multipliers and decay factors the subproblem just updated.
  * A cap max_outer on the iterations (the paper has none).
  * With mu_f > 0 the friction set of Appendix A is captured once, at x^t from
    the incoming constraints and multipliers, and held for the whole step.
"""
from __future__ import annotations

import numpy as np

from . import ccd
from . import friction
from . import subproblem as sp


def time_step(scene, K_min=2, eps=1e-3, max_outer=200, Gamma=0.9, max_newton=20, mu_init_C=None,
              sep=ccd.S_SEP, mu_f=0.0, eps_v=1e-3):
    """Algorithm 1 from scene["x"] (= x^t) and scene["x_hat"] (= x_hat^[0]).
    Returns (x, v, constraints (pt, ee, lam, gam), info)."""
    sc = dict(scene)
    x_t = sc["x"].copy()
    x = x_t.copy()
    xh = sc["x_hat"].copy()
    pt = np.asarray(sc["pt"], dtype=np.int64).reshape(-1, 4)
    ee = np.asarray(sc["ee"], dtype=np.int64).reshape(-1, 4)
    lam = np.asarray(sc["lam"], dtype=np.float64).copy()
    gam = np.asarray(sc["gamma"], dtype=np.float64).copy()
    kappa, delta = float(sc["kappa"]), float(sc["delta"])
    sc["friction"] = friction.capture(sc, mu_f, eps_v) if mu_f > 0 else None
    if mu_init_C is not None:
        kappa = sp.mu_init(sc, mu_init_C)
    tris, edges, verts = ccd.surface(sc["tets"])
    beta, k, stall, doublings = 1.0, 0, 0, 0
    alphas = []
    while beta > eps and k < max_outer:
        cur = dict(sc, x=x, x_hat=xh, pt=pt, ee=ee, lam=lam, gamma=gam, kappa=kappa, delta=delta)
        xh_new, lam, gam, _ = sp.solve_subproblem(cur, max_newton=max_newton, Gamma=Gamma)
        pt, ee, lam, gam, _ = ccd.update_active_set(len(x), x, xh, tris, edges, verts, pt, ee, lam, gam, delta, sep)
        alpha = ccd.max_step_size(x, xh_new, sc["tets"], tris, edges, verts, delta, sep)
        x = (1.0 - alpha) * x + alpha * xh_new
        xh = xh_new
        alphas.append(alpha)
        if k + 1 >= K_min:
            beta *= 1.0 - alpha
        stall = stall + 1 if alpha < 1e-4 else 0
        if stall >= 50:
            kappa, delta, stall = 2.0 * kappa, 0.5 * delta, 0
            doublings += 1
        k += 1
    info = dict(outer=k, beta=beta, alphas=alphas, kappa=kappa, delta=delta, doublings=doublings)
    return x, (x - x_t) / sc["dt"], (pt, ee, lam, gam), info
