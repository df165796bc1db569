"""Plain FP64 CPU oracle for one Newton step of the barrier-free AL contact solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module:
it is used by the tests, by the package smoke check, and by the benchmark's
CPU-baseline leg.  It shares no code with the GPU path.

What it computes (paper: "Augmented Lagrangian-based Subproblem Solver", the
Newton loop of Algorithm 2, and Section 3 for the incremental potential):

  G = grad_x E(x_hat, x_tilde) + sum_i mu*gamma_i*(c_i - lambda_i/mu - s_i) grad d_i(x)
  H = SPDProject(hess E) + sum_i mu*gamma_i grad d_i(x) grad d_i(x)^T
  p* = -H^{-1} G

with E(x) = 1/2 (x - x_tilde)^T M (x - x_tilde) + h^2 U(x) (Section 3, incremental
potential), linearized constraints c_i(x_hat) = d_i(x) + grad d_i(x)^T (x_hat - x)
- delta (Section 4.2, constraint linearization), slacks s_i = max(0, c_i -
lambda_i/mu) (Section 4.2, alternating primal solve), penalty mu (called kappa
by the C-ABI) and moving Dirichlet nodes eliminated by zeroing their gradient
entries and their Hessian rows/columns except the diagonals (Section 5.3).

Everything is a direct definition: the 9x9 Hessian of the energy density is
built column by column from the directional derivative of P, projected by a
library eigendecomposition with eigenvalues clamped at zero (Section 5.1,
SPD projection), and mapped to 12x12 by the dense matrix that sends vertex
displacements to dF.  No analytic eigensystem, no slot maps and no PCG are
used to form G, H or p*.

Readings of points the paper leaves open are listed in the design doc and restated
at the function they affect.  Every function here is pinned by CPU tests.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg
import scipy.sparse as sp
import scipy.sparse.linalg as spla

# Local vertex-pair order of the ten 3x3 blocks of a 4-vertex stencil.
PAIRS = [(0, 0), (0, 1), (0, 2), (0, 3), (1, 1), (1, 2), (1, 3), (2, 2), (2, 3), (3, 3)]


# ---------------------------------------------------------------- geometry ---

def rest_geometry(rest, tets):
    """Dm^{-1}, rest volume and the four row vectors A_a of each tet.

    Dm = [X1-X0, X2-X0, X3-X0] (columns).  F = Ds Dm^{-1}, so dF = dx_a (outer)
    A_a with A_a = row a-1 of Dm^{-1} for a = 1..3 and A_0 = -(A_1+A_2+A_3):
    these are the constant row vectors the paper precomputes per element
    (Section 5.1, vertex-block assembly).
    """
    X = rest[tets]                                   # [T,4,3]
    Dm = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)
    Dminv = np.linalg.inv(Dm)
    vol = np.abs(np.linalg.det(Dm)) / 6.0
    A = np.empty((len(tets), 4, 3))
    A[:, 1:4, :] = Dminv
    A[:, 0, :] = -Dminv.sum(axis=1)
    return Dminv, vol, A


def lame(E, nu):
    """Lame parameters of an isotropic material."""
    mu = E / (2.0 * (1.0 + nu))
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    return mu, lam


def lumped_mass(n_nodes, tets, vol, rho):
    """Diagonal lumped mass (Section 3): each tet gives rho*V/4 to each of its vertices."""
    m = np.zeros(n_nodes)
    np.add.at(m, tets.ravel(), np.repeat(rho * vol / 4.0, 4))
    return m


def deformation_gradient(xh, tets, Dminv):
    P = xh[tets]
    Ds = np.stack([P[:, 1] - P[:, 0], P[:, 2] - P[:, 0], P[:, 3] - P[:, 0]], axis=2)
    return Ds @ Dminv


# --------------------------------------------------------- Neo-Hookean ------
# Reading: the paper names Neo-Hookean without printing it; we take the classic
# compressible form with ln J, which has zero energy and stress at rest.

def nh_energy(F, mu, lam):
    """Psi = mu/2 (tr F^T F - 3) - mu ln J + lam/2 (ln J)^2 per element."""
    J = np.linalg.det(F)
    if np.any(J <= 0):
        raise ValueError("inverted element (J <= 0)")
    lnJ = np.log(J)
    I1 = np.einsum("tij,tij->t", F, F)
    return 0.5 * mu * (I1 - 3.0) - mu * lnJ + 0.5 * lam * lnJ ** 2


def nh_stress(F, mu, lam):
    """First Piola-Kirchhoff stress P = mu (F - F^{-T}) + lam ln J F^{-T}."""
    J = np.linalg.det(F)
    if np.any(J <= 0):
        raise ValueError("inverted element (J <= 0)")
    FinvT = np.transpose(np.linalg.inv(F), (0, 2, 1))
    lnJ = np.log(J)
    return mu[:, None, None] * (F - FinvT) + (lam * lnJ)[:, None, None] * FinvT


def nh_dP(F, dF, mu, lam):
    """Directional derivative of P along dF:
    mu dF + (mu - lam ln J) F^{-T} dF^T F^{-T} + lam tr(F^{-1} dF) F^{-T}."""
    J = np.linalg.det(F)
    lnJ = np.log(J)
    Finv = np.linalg.inv(F)
    FinvT = np.transpose(Finv, (0, 2, 1))
    dFT = np.transpose(dF, (0, 2, 1))
    tr = np.einsum("tij,tji->t", Finv, dF)
    return (mu[:, None, None] * dF
            + (mu - lam * lnJ)[:, None, None] * (FinvT @ dFT @ FinvT)
            + (lam * tr)[:, None, None] * FinvT)


# Stable Neo-Hookean (reading: the rest-stable form of Smith, de Goes and Kim,
# "Analytic Eigensystems for Isotropic Distortion Energies", 2019; the paper
# names SNH in Table 2 without printing it):
#   Psi = mu/2 (tr F^T F - 3) - mu (J - 1) + lam/2 (J - 1)^2.

def snh_energy(F, mu, lam):
    J = np.linalg.det(F)
    I1 = np.einsum("tij,tij->t", F, F)
    return 0.5 * mu * (I1 - 3.0) - mu * (J - 1.0) + 0.5 * lam * (J - 1.0) ** 2


def _cof(F):
    """Cofactor matrix dJ/dF = J F^{-T}."""
    J = np.linalg.det(F)
    return J[:, None, None] * np.transpose(np.linalg.inv(F), (0, 2, 1))


def snh_stress(F, mu, lam):
    """P = mu F + (lam (J - 1) - mu) cof(F)."""
    J = np.linalg.det(F)
    return mu[:, None, None] * F + (lam * (J - 1.0) - mu)[:, None, None] * _cof(F)


def snh_dP(F, dF, mu, lam):
    """mu dF + lam (cof F : dF) cof F + (lam (J - 1) - mu) d(cof F)[dF], with
    d(cof F)[dF] = J (tr(F^{-1} dF) F^{-T} - F^{-T} dF^T F^{-T})."""
    J = np.linalg.det(F)
    Finv = np.linalg.inv(F)
    FinvT = np.transpose(Finv, (0, 2, 1))
    C = J[:, None, None] * FinvT
    dFT = np.transpose(dF, (0, 2, 1))
    tr = np.einsum("tij,tji->t", Finv, dF)
    dC = J[:, None, None] * (tr[:, None, None] * FinvT - FinvT @ dFT @ FinvT)
    return (mu[:, None, None] * dF + (lam * np.einsum("tij,tij->t", C, dF))[:, None, None] * C
            + (lam * (J - 1.0) - mu)[:, None, None] * dC)


# Corotated linear elasticity (reading: Table 2's "corotated linear (COR)"; the
# classic form built on the polar decomposition F = R S, R a rotation and S
# symmetric): Psi = mu ||F - R||^2 + lam/2 (tr S - 3)^2, i.e. linear elasticity
# in the corotated frame, in terms of S - I.

def polar(F):
    """F = R S with det R = +1 (from a library SVD: R = U V^T with the sign of
    the smallest singular direction flipped when det F < 0)."""
    U, s, Vt = np.linalg.svd(F)
    d = np.sign(np.linalg.det(U @ Vt))
    U = U.copy()
    U[:, :, 2] *= d[:, None]
    R = U @ Vt
    S = np.transpose(R, (0, 2, 1)) @ F
    return R, 0.5 * (S + np.transpose(S, (0, 2, 1)))


def cor_energy(F, mu, lam):
    R, S = polar(F)
    trS = np.einsum("tii->t", S)
    return mu * np.einsum("tij,tij->t", F - R, F - R) + 0.5 * lam * (trS - 3.0) ** 2


def cor_stress(F, mu, lam):
    """P = 2 mu (F - R) + lam (tr S - 3) R: the rotation's variation drops out,
    since (F - R) : dR = (S - I) : R^T dR and R^T dR is skew."""
    R, S = polar(F)
    trS = np.einsum("tii->t", S)
    return 2.0 * mu[:, None, None] * (F - R) + (lam * (trS - 3.0))[:, None, None] * R


def _polar_rotation_differential(R, S, dF):
    """dR = R [w]x with (tr S I - S) w = axial(R^T dF - dF^T R): from
    R^T dF = (R^T dR) S + dS with R^T dR skew and dS symmetric, the skew part
    gives W S + S W = R^T dF - dF^T R, and W S + S W = [(tr S I - S) w]x."""
    A = np.transpose(R, (0, 2, 1)) @ dF
    A = A - np.transpose(A, (0, 2, 1))
    a = np.stack([A[:, 2, 1], A[:, 0, 2], A[:, 1, 0]], axis=1)
    M = np.einsum("tii->t", S)[:, None, None] * np.eye(3)[None] - S
    w = np.linalg.solve(M, a[:, :, None])[:, :, 0]
    W = np.zeros_like(R)
    W[:, 0, 1], W[:, 0, 2], W[:, 1, 2] = -w[:, 2], w[:, 1], -w[:, 0]
    W[:, 1, 0], W[:, 2, 0], W[:, 2, 1] = w[:, 2], -w[:, 1], w[:, 0]
    return R @ W


def cor_dP(F, dF, mu, lam):
    """2 mu (dF - dR) + lam (R : dF) R + lam (tr S - 3) dR, using
    d tr S = R : dF."""
    R, S = polar(F)
    trS = np.einsum("tii->t", S)
    dR = _polar_rotation_differential(R, S, dF)
    RdF = np.einsum("tij,tij->t", R, dF)
    return (2.0 * mu[:, None, None] * (dF - dR) + (lam * RdF)[:, None, None] * R
            + (lam * (trS - 3.0))[:, None, None] * dR)


# Materials per tet: 0 Neo-Hookean, 1 stable Neo-Hookean, 2 corotated linear.
# Every energy needs J > 0 here (the solver keeps every tet uninverted).

def _mat(mat, T):
    return np.zeros(T, dtype=np.int64) if mat is None else np.asarray(mat, dtype=np.int64)


def psi_energy(F, mu, lam, mat=None):
    m = _mat(mat, len(F))
    J = np.linalg.det(F)
    if np.any(J <= 0):
        raise ValueError("inverted element (J <= 0)")
    out = np.empty(len(F))
    for code, fn in ((0, nh_energy), (1, snh_energy), (2, cor_energy)):
        k = m == code
        if k.any():
            out[k] = fn(F[k], mu[k], lam[k])
    return out


def psi_stress(F, mu, lam, mat=None):
    m = _mat(mat, len(F))
    out = np.empty_like(F)
    for code, fn in ((0, nh_stress), (1, snh_stress), (2, cor_stress)):
        k = m == code
        if k.any():
            out[k] = fn(F[k], mu[k], lam[k])
    return out


def psi_dP(F, dF, mu, lam, mat=None):
    m = _mat(mat, len(F))
    out = np.empty_like(F)
    for code, fn in ((0, nh_dP), (1, snh_dP), (2, cor_dP)):
        k = m == code
        if k.any():
            out[k] = fn(F[k], dF[k], mu[k], lam[k])
    return out


def nh_hessian9(F, mu, lam, mat=None):
    """d^2 Psi / dF^2 as a 9x9 matrix over row-major vec(F) (index 3i+j <-> F_ij),
    built column by column from the directional derivative, then symmetrized
    (per tet of its material; Neo-Hookean when mat is None)."""
    T = len(F)
    H = np.empty((T, 9, 9))
    for k in range(9):
        E = np.zeros((T, 3, 3))
        E[:, k // 3, k % 3] = 1.0
        H[:, :, k] = psi_dP(F, E, mu, lam, mat).reshape(T, 9)
    return 0.5 * (H + np.transpose(H, (0, 2, 1)))


def psd_project(H):
    """Clamp the eigenvalues of each symmetric matrix at zero (Section 5.1:
    omega_k^+ = max(omega_k, 0)); eigendecomposition by LAPACK."""
    w, Q = np.linalg.eigh(H)
    w = np.maximum(w, 0.0)
    return (Q * w[:, None, :]) @ np.transpose(Q, (0, 2, 1))


def dF_map(A):
    """B [T,9,12]: vec(dF) = B x_e with x_e = (x_0, x_1, x_2, x_3) vertex-major.
    dF_ij = sum_a dx_{a,i} A_{a,j}, so B[3i+j, 3a+i] = A_{a,j}."""
    T = len(A)
    B = np.zeros((T, 9, 12))
    for a in range(4):
        for i in range(3):
            for j in range(3):
                B[:, 3 * i + j, 3 * a + i] = A[:, a, j]
    return B


def elastic_terms(xh, tets, Dminv, vol, A, mu, lam, h, mat=None):
    """Per-element gradient h^2 V P A_a^T [T,4,3] and PSD-projected Hessian
    h^2 V B^T (d2Psi/dF2)^+ B [T,12,12]."""
    F = deformation_gradient(xh, tets, Dminv)
    if np.any(np.linalg.det(F) <= 0):
        raise ValueError("inverted element (J <= 0)")
    P = psi_stress(F, mu, lam, mat)
    w = h * h * vol
    g = w[:, None, None] * np.einsum("tij,taj->tai", P, A)
    H9p = psd_project(nh_hessian9(F, mu, lam, mat))
    B = dF_map(A)
    He = w[:, None, None] * (np.transpose(B, (0, 2, 1)) @ H9p @ B)
    return g, He


# ------------------------------------------------------------- distances ----
# Reading: d_i is the unsigned Euclidean distance between the closed primitives
# (Section 3), a function of all 12 coordinates; its gradient is w (outer) n
# with n the unit vector from the second primitive's closest point to the first's.

def _seg_param(p, u, v):
    """Parameter of the point of segment [u, v] closest to p, clamped to [0,1]."""
    e = v - u
    return np.clip(np.einsum("ij,ij->i", p - u, e) / np.einsum("ij,ij->i", e, e), 0.0, 1.0)


def pt_closest(p, t0, t1, t2):
    """Closest point of the closed triangle (t0,t1,t2) to p.

    Returns (d, n, w) with d = |p - q|, n = (p - q)/d and w = (1, -b0, -b1, -b2)
    where q = b0 t0 + b1 t1 + b2 t2.  The closest point is the orthogonal
    projection when it lies inside the triangle, else the closest of the three
    edge points.
    """
    n = len(p)
    e1, e2, r = t1 - t0, t2 - t0, p - t0
    a11 = np.einsum("ij,ij->i", e1, e1)
    a12 = np.einsum("ij,ij->i", e1, e2)
    a22 = np.einsum("ij,ij->i", e2, e2)
    r1 = np.einsum("ij,ij->i", e1, r)
    r2 = np.einsum("ij,ij->i", e2, r)
    det = a11 * a22 - a12 * a12
    u = (a22 * r1 - a12 * r2) / det
    v = (a11 * r2 - a12 * r1) / det
    inside = (u >= 0) & (v >= 0) & (u + v <= 1)
    cands = []  # (dist, barycentrics [n,3])
    bi = np.stack([1 - u - v, u, v], axis=1)
    qi = t0 + u[:, None] * e1 + v[:, None] * e2
    di = np.where(inside, np.linalg.norm(p - qi, axis=1), np.inf)
    cands.append((di, bi))
    for (ia, ib) in ((0, 1), (1, 2), (2, 0)):
        T = (t0, t1, t2)
        s = _seg_param(p, T[ia], T[ib])
        q = T[ia] + s[:, None] * (T[ib] - T[ia])
        b = np.zeros((n, 3))
        b[:, ia] = 1 - s
        b[:, ib] = s
        cands.append((np.linalg.norm(p - q, axis=1), b))
    D = np.stack([c[0] for c in cands], axis=1)
    k = np.argmin(D, axis=1)
    bary = np.stack([c[1] for c in cands], axis=1)[np.arange(n), k]
    q = bary[:, 0:1] * t0 + bary[:, 1:2] * t1 + bary[:, 2:3] * t2
    diff = p - q
    d = np.linalg.norm(diff, axis=1)
    nrm = diff / d[:, None]
    w = np.column_stack([np.ones(n), -bary])
    return d, nrm, w


def ee_closest(a0, a1, b0, b1):
    """Closest points of segments a0 + s(a1-a0) and b0 + t(b1-b0), (s,t) in [0,1]^2.

    Returns (d, n, w) with n = (P - Q)/d and w = (1-s, s, -(1-t), -t).  The
    minimizer is the interior stationary point when it lies in the square,
    else the best of the four edge-clamped candidates.
    """
    n = len(a0)
    ea, eb, r = a1 - a0, b1 - b0, a0 - b0
    aa = np.einsum("ij,ij->i", ea, ea)
    bb = np.einsum("ij,ij->i", eb, eb)
    ab = np.einsum("ij,ij->i", ea, eb)
    ar = np.einsum("ij,ij->i", ea, r)
    br = np.einsum("ij,ij->i", eb, r)
    # stationarity of |r + s ea - t eb|^2:  aa s - ab t = -ar ;  ab s - bb t = -br
    det = aa * bb - ab * ab
    with np.errstate(divide="ignore", invalid="ignore"):
        s_in = (-ar * bb + ab * br) / det
        t_in = (aa * br - ab * ar) / det
    inside = (det > 0) & (s_in >= 0) & (s_in <= 1) & (t_in >= 0) & (t_in <= 1)
    S, Tt, D = [], [], []

    def add(s, t, valid=None):
        P = a0 + s[:, None] * ea
        Q = b0 + t[:, None] * eb
        d = np.linalg.norm(P - Q, axis=1)
        if valid is not None:
            d = np.where(valid, d, np.inf)
        S.append(s)
        Tt.append(t)
        D.append(d)

    add(np.where(inside, s_in, 0.0), np.where(inside, t_in, 0.0), inside)
    zero, one = np.zeros(n), np.ones(n)
    add(zero, _seg_param(a0, b0, b1))
    add(one, _seg_param(a1, b0, b1))
    add(_seg_param(b0, a0, a1), zero)
    add(_seg_param(b1, a0, a1), one)
    D = np.stack(D, axis=1)
    k = np.argmin(D, axis=1)
    s = np.stack(S, axis=1)[np.arange(n), k]
    t = np.stack(Tt, axis=1)[np.arange(n), k]
    diff = (a0 + s[:, None] * ea) - (b0 + t[:, None] * eb)
    d = np.linalg.norm(diff, axis=1)
    nrm = diff / d[:, None]
    w = np.column_stack([1 - s, s, -(1 - t), -t])
    return d, nrm, w


def linearize(x, pt, ee):
    """Distances and gradients of every constraint at the linearization point x
    (Algorithm 2, before the Newton loop).  PT rows are (p, t0, t1, t2), EE rows
    (a0, a1, b0, b1); PT constraints come first.  Returns (ids [n,4], d, n, w)."""
    ids = np.concatenate([pt, ee]).astype(np.int64)
    d = np.empty(len(ids))
    nrm = np.empty((len(ids), 3))
    w = np.empty((len(ids), 4))
    npt = len(pt)
    if npt:
        X = x[pt]
        d[:npt], nrm[:npt], w[:npt] = pt_closest(X[:, 0], X[:, 1], X[:, 2], X[:, 3])
    if len(ee):
        X = x[ee]
        d[npt:], nrm[npt:], w[npt:] = ee_closest(X[:, 0], X[:, 1], X[:, 2], X[:, 3])
    return ids, d, nrm, w


# ------------------------------------------------------------- AL terms -----

def constraint_values(xh, x, ids, d, nrm, w, delta):
    """c_i(x_hat) = d_i(x) + grad d_i(x)^T (x_hat - x) - delta."""
    dx = xh[ids] - x[ids]                                   # [n,4,3]
    return d + np.einsum("na,nak,nk->n", w, dx, nrm) - delta


def al_terms(c, lam_i, gamma, mu, w, nrm):
    """Per-constraint gradient factor and Hessian weight (Algorithm 2, contact loop).

    s_i = max(0, c_i - lambda_i/mu);  G += mu gamma_i (c_i - lambda_i/mu - s_i) grad d_i;
    H += mu gamma_i grad d_i grad d_i^T, kept also when s_i > 0.
    Returns (gfac [n] with G_a += gfac w_a n, hfac [n] with block(a,b) = hfac w_a w_b n n^T).
    """
    s = np.maximum(0.0, c - lam_i / mu)
    gfac = mu * gamma * (c - lam_i / mu - s)
    hfac = mu * gamma
    return gfac, np.broadcast_to(hfac, c.shape).astype(np.float64)


def al_energy(c, lam_i, gamma, mu):
    """gamma (mu/2 (c-s)^2 - lambda (c-s)) with s = max(0, c - lambda/mu)."""
    s = np.maximum(0.0, c - lam_i / mu)
    return gamma * (0.5 * mu * (c - s) ** 2 - lam_i * (c - s))


# --------------------------------------------------------------- assembly ---

class Step:
    """Everything the oracle knows about one Newton step of one scene."""


def prepare(scene):
    """Per-mesh quantities: geometry, Lame parameters, lumped mass."""
    st = Step()
    st.scene = scene
    st.N = len(scene["rest"])
    st.tets = scene["tets"].astype(np.int64)
    st.Dminv, st.vol, st.A = rest_geometry(scene["rest"], st.tets)
    st.mu_l, st.lam_l = lame(scene["E"], scene["nu"])
    st.mat = np.asarray(scene.get("material", np.zeros(len(scene["tets"]))), dtype=np.int64)
    st.mass = lumped_mass(st.N, st.tets, st.vol, scene["rho"])
    st.fixed = scene["fixed"].astype(bool)
    return st


def assemble(scene, st=None):
    """G [N,3] and H (scipy CSR, 3N x 3N, both triangles) after DBC, plus pieces."""
    if st is None:
        st = prepare(scene)
    xh, x, xt, h = scene["x_hat"], scene["x"], scene["x_tilde"], scene["dt"]
    N = st.N
    # inertia: M (x_hat - x_tilde) and M
    G = st.mass[:, None] * (xh - xt)
    rows, cols, vals = [], [], []
    diag = np.arange(3 * N)
    rows.append(diag)
    cols.append(diag)
    vals.append(np.repeat(st.mass, 3))
    # elasticity
    ge, He = elastic_terms(xh, st.tets, st.Dminv, st.vol, st.A, st.mu_l, st.lam_l, h, st.mat)
    np.add.at(G, st.tets.ravel(), ge.reshape(-1, 3))
    dof = (3 * st.tets[:, :, None] + np.arange(3)[None, None, :]).reshape(-1, 12)
    rows.append(np.repeat(dof, 12, axis=1).ravel())
    cols.append(np.tile(dof, (1, 12)).ravel())
    vals.append(He.ravel())
    # augmented-Lagrangian contact terms
    ids, d, nrm, w = linearize(x, scene["pt"], scene["ee"])
    c = constraint_values(xh, x, ids, d, nrm, w, scene["delta"])
    gfac, hfac = al_terms(c, scene["lam"], scene["gamma"], scene["kappa"], w, nrm)
    grad = w[:, :, None] * nrm[:, None, :]                 # [n,4,3] = grad d_i
    np.add.at(G, ids.ravel(), (gfac[:, None, None] * grad).reshape(-1, 3))
    gv = grad.reshape(-1, 12)
    Hc = hfac[:, None, None] * gv[:, :, None] * gv[:, None, :]
    cdof = (3 * ids[:, :, None] + np.arange(3)[None, None, :]).reshape(-1, 12)
    rows.append(np.repeat(cdof, 12, axis=1).ravel())
    cols.append(np.tile(cdof, (1, 12)).ravel())
    vals.append(Hc.ravel())
    # semi-implicit friction of the previous step's contacts (Appendix A)
    if scene.get("friction") is not None:
        from . import friction
        friction.add_to(scene["friction"], xh, G, rows, cols, vals)
    H = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(3 * N, 3 * N)).tocsr()
    H.sum_duplicates()
    G, H = apply_dbc(G, H, st.fixed)
    st.G, st.H = G, H
    st.ids, st.d, st.nrm, st.w, st.c = ids, d, nrm, w, c
    st.gfac, st.hfac = gfac, hfac
    return st


def apply_dbc(G, H, fixed):
    """Section 5.3: zero the gradient of fixed nodes and every Hessian entry in
    their rows and columns except the scalar diagonals."""
    if not fixed.any():
        return G, H
    G = G.copy()
    G[fixed] = 0.0
    fd = np.repeat(fixed, 3)
    keep = sp.diags((~fd).astype(np.float64))
    Hd = H.diagonal()
    H = keep @ H @ keep + sp.diags(np.where(fd, Hd, 0.0))
    return G, H.tocsr()


def total_energy(scene, st, xh):
    """L(x_hat) = 1/2 |x_hat - x_tilde|_M^2 + h^2 sum V Psi + sum AL terms
    (Section 4.2, total energy), plus the friction terms when the scene holds a
    friction set (Appendix A).  Used only to check G by finite differences."""
    h = scene["dt"]
    F = deformation_gradient(xh, st.tets, st.Dminv)
    Ei = 0.5 * np.sum(st.mass[:, None] * (xh - scene["x_tilde"]) ** 2)
    Ee = h * h * np.sum(st.vol * psi_energy(F, st.mu_l, st.lam_l, st.mat))
    ids, d, nrm, w = linearize(scene["x"], scene["pt"], scene["ee"])
    c = constraint_values(xh, scene["x"], ids, d, nrm, w, scene["delta"])
    Ec = np.sum(al_energy(c, scene["lam"], scene["gamma"], scene["kappa"]))
    Ef = 0.0
    if scene.get("friction") is not None:
        from . import friction
        Ef = friction.energy(scene["friction"], xh)
    return Ei + Ee + Ec + Ef


# ---------------------------------------------------------------- pattern ---

def pattern(n_nodes, tets, pt, ee):
    """Upper 3x3-block pattern of H (Section 5.1: diagonal and upper blocks only).

    Row r holds the sorted unique columns c >= r of {(v, v)} and of (min, max)
    over every vertex pair of every tet and every constraint.  Rows of fixed
    nodes stay in the pattern.  Maps: emap[e][k] / cmap[i][k] is the slot of
    local pair k in PAIRS order (transposed when the first vertex is larger),
    diag[v] is the slot of (v, v).  Returns (row_ptr int64, col int32, emap,
    cmap, diag)."""
    stencils = [np.asarray(tets, dtype=np.int64).reshape(-1, 4)]
    cons = np.concatenate([pt, ee]).astype(np.int64).reshape(-1, 4)
    stencils.append(cons)
    keys = [np.stack([np.arange(n_nodes), np.arange(n_nodes)], axis=1)]
    for S in stencils:
        for (a, b) in PAIRS:
            if a == b:
                continue
            lo = np.minimum(S[:, a], S[:, b])
            hi = np.maximum(S[:, a], S[:, b])
            keys.append(np.stack([lo, hi], axis=1))
    K = np.concatenate(keys)
    key = K[:, 0] * n_nodes + K[:, 1]
    uk = np.unique(key)
    r = uk // n_nodes
    c = uk % n_nodes
    row_ptr = np.zeros(n_nodes + 1, dtype=np.int64)
    np.add.at(row_ptr, r + 1, 1)
    row_ptr = np.cumsum(row_ptr)

    def slots(S):
        out = np.empty((len(S), len(PAIRS)), dtype=np.int64)
        for k, (a, b) in enumerate(PAIRS):
            lo = np.minimum(S[:, a], S[:, b])
            hi = np.maximum(S[:, a], S[:, b])
            out[:, k] = np.searchsorted(uk, lo * n_nodes + hi)
        return out

    emap = slots(stencils[0])
    cmap = slots(cons)
    diag = np.searchsorted(uk, np.arange(n_nodes) * n_nodes + np.arange(n_nodes))
    return row_ptr, c.astype(np.int32), emap, cmap, diag


def upper_blocks(H, row_ptr, col):
    """The 3x3 block of H at every slot of the upper pattern, [nnzb,3,3]."""
    N = len(row_ptr) - 1
    rows = np.repeat(np.arange(N), np.diff(row_ptr))
    Hd = H.tocsr()
    out = np.empty((len(col), 3, 3))
    for i in range(3):
        for j in range(3):
            out[:, i, j] = np.asarray(Hd[3 * rows + i, 3 * col.astype(np.int64) + j]).ravel()
    return out


# ----------------------------------------------------------------- solves ---

def solve_direct(H, G, method="auto"):
    """p* = -H^{-1} G by dense Cholesky (small systems) or SuperLU (sparse)."""
    b = -G.reshape(-1)
    n = H.shape[0]
    if method == "cholesky" or (method == "auto" and n <= 6000):
        c = scipy.linalg.cho_factor(H.toarray())
        p = scipy.linalg.cho_solve(c, b)
    else:
        p = spla.splu(H.tocsc(), permc_spec="COLAMD").solve(b)
    return p.reshape(-1, 3)


def solve_reference(H, G, direct_max_dof=30000):
    """Reference p*: the direct solve up to `direct_max_dof` unknowns, beyond it
    FP64 block-Jacobi PCG to a relative residual of 1e-12 (whose distance to
    the direct solution is pinned by the CPU tests)."""
    if H.shape[0] <= direct_max_dof:
        return solve_direct(H, G)
    p, _ = block_jacobi_pcg(H, G, 1e-12, max_iter=200000)
    return p


def block_jacobi_pcg(H, G, tol, max_iter=20000, record=None):
    """FP64 PCG on H p = -G with the 3x3 block-Jacobi preconditioner, x0 = 0,
    stopping at |r|_2 <= tol |b|_2 (the paper's CG relative tolerance).

    `record`, a dict keyed by looser tolerances, receives (iterate, iterations)
    the first time the residual meets each of them: the solve at that
    tolerance, since the iterates do not depend on where the loop stops."""
    b = -G.reshape(-1)
    n = H.shape[0]
    N = n // 3
    Hc = H.tocsr()
    D = np.empty((N, 3, 3))
    idx = np.arange(N)
    for i in range(3):
        for j in range(3):
            D[:, i, j] = np.asarray(Hc[3 * idx + i, 3 * idx + j]).ravel()
    Dinv = np.linalg.inv(D)

    def prec(r):
        return np.einsum("nij,nj->ni", Dinv, r.reshape(N, 3)).reshape(-1)

    x = np.zeros(n)
    r = b.copy()
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return x.reshape(-1, 3), 0
    z = prec(r)
    p = z.copy()
    rz = r @ z
    it = 0
    pending = sorted(record, reverse=True) if record is not None else []
    while True:
        rn = np.linalg.norm(r)
        while pending and rn <= pending[0] * bn:
            record[pending.pop(0)] = (x.reshape(-1, 3).copy(), it)
        if not (rn > tol * bn and it < max_iter):
            break
        q = Hc @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        z = prec(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
        it += 1
    return x.reshape(-1, 3), it


def energy_norm_rel(H, p, p_ref):
    """|p - p_ref|_H / |p_ref|_H."""
    e = (p - p_ref).reshape(-1)
    r = p_ref.reshape(-1)
    return float(np.sqrt(e @ (H @ e)) / np.sqrt(r @ (H @ r)))


def stats(scene, st, p):
    """|p|_inf / h and max_i max(0, -c_i(x_hat)) (FP64)."""
    return dict(newton_inf_over_h=float(np.abs(p).max() / scene["dt"]),
                max_violation=float(np.maximum(0.0, -st.c).max()) if len(st.c) else 0.0)
