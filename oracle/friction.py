"""Plain FP64 CPU oracle for the semi-implicit friction of Appendix A.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Appendix A adds the smoothed friction potential of IPC (Li et al. 2020) to
U(x):  U_f(x) = sum_i mu_f F_i^t f_0(|u_i|; eps_v),  over the active contacts
of the previous time step, with F_i^t the normal force there and u_i the
tangential relative displacement.  The total energy holds h^2 U(x), and the
normal force is F_i^t = h^-2 kappa (lambda_i / kappa + s_i - c_i(x^t)) in
magnitude, so each contact contributes

    coef_i f_0(|u_i|),   coef_i = mu_f max(0, lambda_i - kappa c_i(x^t)),

(the slack's minimizer makes lambda + kappa (s - c) = max(0, lambda - kappa c)).
Semi-implicit: the contact's closest-point weights w, normal n and coef are
taken at x^t and held for the whole step; u_i = P_i sum_a w_a (x_a - x^t_a)
with P_i = I - n n^T the projection onto the contact's tangent plane (the IPC
form T^T (.) with an orthonormal tangent basis T gives the same |u| and,
mapped back by T, the same gradient and Hessian).

f_0 (IPC): f_0(y) = y for y >= eps_v h, and -y^3/(3 e^2) + y^2/e + e/3 with
e = eps_v h below, which makes f_0 twice continuously differentiable; its
derivative is f_1(y) = 1 above and 2y/e - y^2/e^2 below.

Readings (listed in the design doc): the force's magnitude max(0, lambda - kappa c)
(Appendix A prints the signed expression), c_i(x^t) the exact distance at
x^t minus delta, and the per-contact Hessian projected onto the SPD cone
(Section 5.1), which leaves it unchanged since f_0 of a norm is convex.
"""
from __future__ import annotations

import numpy as np

from . import core


def f0(y, e):
    y = np.asarray(y, dtype=np.float64)
    return np.where(y >= e, y, -y ** 3 / (3.0 * e * e) + y * y / e + e / 3.0)


def f1(y, e):
    """f_0'(y)."""
    y = np.asarray(y, dtype=np.float64)
    return np.where(y >= e, 1.0, 2.0 * y / e - y * y / (e * e))


def f1_prime(y, e):
    """f_0''(y)."""
    y = np.asarray(y, dtype=np.float64)
    return np.where(y >= e, 0.0, 2.0 / e - 2.0 * y / (e * e))


def capture(scene, mu_f, eps_v):
    """The friction set of a time step from the constraints of the previous one
    (scene["pt"], ["ee"], ["lam"]) at x^t = scene["x"]."""
    x, h = scene["x"], scene["dt"]
    ids, d, nrm, w = core.linearize(x, np.asarray(scene["pt"]).reshape(-1, 4), np.asarray(scene["ee"]).reshape(-1, 4))
    c = d - scene["delta"]
    force = np.maximum(0.0, np.asarray(scene["lam"], dtype=np.float64) - scene["kappa"] * c) / (h * h)
    return dict(ids=ids, nrm=nrm, w=w, coef=h * h * mu_f * force, x0=x.copy(), e=eps_v * h)


def _tangent(fr, xh):
    v = np.einsum("ia,iak->ik", fr["w"], xh[fr["ids"]] - fr["x0"][fr["ids"]])
    n = fr["nrm"]
    ut = v - np.einsum("ik,ik->i", n, v)[:, None] * n
    return ut, np.linalg.norm(ut, axis=1)


def energy(fr, xh):
    """sum_i coef_i f_0(|u_i|)."""
    if len(fr["ids"]) == 0:
        return 0.0
    _, y = _tangent(fr, xh)
    return float(np.sum(fr["coef"] * f0(y, fr["e"])))


def terms(fr, xh):
    """Per contact the gradient of coef f_0(|u|) with respect to the relative
    displacement v = sum_a w_a (x_a - x^t_a), and its Hessian projected onto the
    SPD cone: grad = coef f_1(y)/y u, hess = coef (f_1(y)/y P + (f_1'(y) -
    f_1(y)/y) t t^T) with t = u / y (at y = 0 the limit coef (2/e) P)."""
    ut, y = _tangent(fr, xh)
    e = fr["e"]
    n = fr["nrm"]
    P = np.eye(3)[None] - n[:, :, None] * n[:, None, :]
    safe = np.where(y > 0.0, y, 1.0)
    f1_over_y = np.where(y >= e, 1.0 / safe, 2.0 / e - y / (e * e))
    t = ut / safe[:, None]
    gv = (fr["coef"] * f1_over_y)[:, None] * ut
    Hv = f1_over_y[:, None, None] * P + (f1_prime(y, e) - f1_over_y)[:, None, None] * (t[:, :, None] * t[:, None, :])
    Hv = core.psd_project(fr["coef"][:, None, None] * Hv)
    return gv, Hv


def add_to(fr, xh, G, rows, cols, vals):
    """Scatter the friction gradient into G [N,3] and the 12x12 Hessian blocks
    w_a w_b Hv into COO lists."""
    if len(fr["ids"]) == 0:
        return
    gv, Hv = terms(fr, xh)
    ids, w = fr["ids"], fr["w"]
    np.add.at(G, ids.ravel(), (w[:, :, None] * gv[:, None, :]).reshape(-1, 3))
    blk = w[:, :, None, None, None] * w[:, None, :, None, None] * Hv[:, None, None, :, :]   # [n,a,b,3,3]
    H12 = np.transpose(blk, (0, 1, 3, 2, 4)).reshape(-1, 12, 12)
    dof = (3 * ids[:, :, None] + np.arange(3)[None, None, :]).reshape(-1, 12)
    rows.append(np.repeat(dof, 12, axis=1).ravel())
    cols.append(np.tile(dof, (1, 12)).ravel())
    vals.append(H12.ravel())
