"""Plain FP64 CPU oracle for the rest of SolveSubproblem (Algorithm 2).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Algorithm 2 (Section 4.2, "Alternating Primal Solve"): with the distances
linearized once at the intersection-free state x, repeat projected Newton
steps on x_hat -- gradient and SPD-projected Hessian of the total energy L,
p = -H^{-1} G, a line search for 0 <= r <= 1 with L(x_hat + r p) < L(x_hat),
x_hat += r p -- until a full step (r = 1) is taken; then update every
constraint's multiplier and decay factor from its slack s_i = max(0, c_i -
lambda_i/mu): when s_i = 0, lambda_i -= mu c_i and gamma_i = 1, otherwise
lambda_i = 0 and gamma_i *= Gamma (Section 4.2, "Constraint Decay",
Gamma = 0.9).  Section 5.2 sets the penalty at the start of a time step to
C max_i (grad^2 E)_ii with C = 0.1.

Readings (listed in the design doc):
  * L is the total energy of Section 4.2 with each slack at its minimizer
    s_i = max(0, c_i - lambda_i/mu), the value the Newton step uses; so L is a
    function of x_hat alone (core.total_energy) and G is its gradient.
  * The line search is backtracking by halving from r = 1, taking the first r
    with L(x_hat + r p) < L(x_hat); a state with an inverted element has
    infinite energy (Neo-Hookean is non-invertible).  After 30 halvings the
    step is r = 0 and the loop stops.
  * The Newton loop stops after max_newton steps even without a full step.
  * The penalty estimate of Section 5.2 takes the diagonal of the Hessian the
    solver assembles (lumped mass plus SPD-projected elasticity) at x, the
    state the time step starts from.
Each step uses the direct solve of core.solve_direct (the exact Newton step).
"""
from __future__ import annotations

import numpy as np

from . import core


def energy(scene, st, xh):
    """L(x_hat) in FP64, +inf for a state with an inverted element."""
    try:
        return core.total_energy(scene, st, xh)
    except ValueError:
        return np.inf


def line_search(scene, st, xh, p, L0, max_halvings=30):
    """Backtracking by halving: the first r = 2^-k (k = 0, 1, ...) with
    L(x_hat + r p) < L0.  Returns (r, L(x_hat + r p)); (0, L0) if none."""
    r = 1.0
    for _ in range(max_halvings + 1):
        L = energy(scene, st, xh + r * p)
        if L < L0:
            return r, L
        r *= 0.5
    return 0.0, L0


def constraint_values_at(scene, xh):
    """c_i(x_hat) with the distances linearized at x (Section 4.2)."""
    ids, d, nrm, w = core.linearize(scene["x"], scene["pt"], scene["ee"])
    return core.constraint_values(xh, scene["x"], ids, d, nrm, w, scene["delta"])


def dual_update(scene, xh, Gamma=0.9):
    """Multiplier and decay update after the Newton loop of Algorithm 2.
    Returns (lambda', gamma', active) with active_i = (s_i == 0)."""
    mu = scene["kappa"]
    lam, gam = scene["lam"], scene["gamma"]
    c = constraint_values_at(scene, xh)
    s = np.maximum(0.0, c - lam / mu)
    active = s == 0.0
    lam_new = np.where(active, lam - mu * c, 0.0)
    gam_new = np.where(active, 1.0, Gamma * gam)
    return lam_new, gam_new, active


def hessian_diagonal(scene, st, xs):
    """The 3N scalar diagonal of the incremental potential's Hessian at xs:
    the lumped mass plus the diagonal of every element's SPD-projected
    h^2 V B^T (d2Psi/dF2)^+ B (the matrix the Newton step assembles)."""
    diag = np.repeat(st.mass, 3).astype(np.float64)
    _, He = core.elastic_terms(xs, st.tets, st.Dminv, st.vol, st.A, st.mu_l, st.lam_l, scene["dt"], st.mat)
    dof = (3 * st.tets[:, :, None] + np.arange(3)[None, None, :]).reshape(-1, 12)
    np.add.at(diag, dof.ravel(), np.diagonal(He, axis1=1, axis2=2).ravel())
    return diag


def mu_init(scene, C=0.1, st=None):
    """Section 5.2: the initial penalty C max_i (grad^2 E)_ii, taken at x, the
    state the time step starts from."""
    st = core.prepare(scene) if st is None else st
    return C * float(hessian_diagonal(scene, st, scene["x"]).max())


def solve_subproblem(scene, max_newton=50, Gamma=0.9):
    """Algorithm 2 from scene["x_hat"]: returns (x_hat, lambda', gamma', history)
    with history = [(L before the step, r, L after)] per Newton step."""
    xh = scene["x_hat"].copy()
    prep = core.prepare(scene)
    hist = []
    for _ in range(max_newton):
        sc = dict(scene)
        sc["x_hat"] = xh
        st = core.assemble(sc, core.prepare(scene))
        p = core.solve_direct(st.H, st.G)
        L0 = energy(scene, prep, xh)
        r, L1 = line_search(scene, prep, xh, p, L0)
        hist.append((L0, r, L1))
        xh = xh + r * p
        if r == 1.0 or r == 0.0:
            break
    lam, gam, _ = dual_update(scene, xh, Gamma)
    return xh, lam, gam, hist
