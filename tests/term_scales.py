"""Per-node and per-block scales for element-wise parity bars.

G and every block of H are sums of terms (inertia, one per tet, one per
constraint).  The GPU rounds each term to FP32 relative to that term's own
size, and the terms of a node or block can cancel, so the right yardstick for
an entry's error is the sum of the magnitudes of the terms it collects, not
the entry itself nor a global norm.  An element's gradient and Hessian are
computed as a whole (one SVD and eigensystem per tet), so a tet's terms are
measured by that tet's whole gradient / 12x12 Hessian.

    gradient_scale[v] = m_v |x_hat_v - x_tilde_v| + sum_{tets e at v} |g_e|
                        + sum_{constraints i at v} |gfac_i| |w_i|
    block_scale[slot] = sum_{tets e at slot} |H_e|_F
                        + sum_{constraints i at slot} hfac_i |w_i|^2
                        + sqrt(3) m_v on the diagonal slot of v

with |grad d_i| = |w_i| (|n| = 1) and |hfac w w^T (x) n n^T|_F = hfac |w|^2.
Dirichlet nodes: their gradient and their off-diagonal blocks are exactly
zero (scale 0).  Test infrastructure: uses the oracle's own per-term
quantities, no GPU output.
"""
import numpy as np

import oracle


def scales(scene, st, row_ptr, col):
    """(gradient_scale [N], block_scale [nnzb]) for the oracle step `st` on the
    upper pattern (row_ptr, col)."""
    N = st.N
    fixed = st.fixed
    ge, He = oracle.elastic_terms(scene["x_hat"], st.tets, st.Dminv, st.vol, st.A, st.mu_l, st.lam_l,
                                  scene["dt"], st.mat)
    T = len(st.tets)
    gs = st.mass * np.linalg.norm(scene["x_hat"] - scene["x_tilde"], axis=1)
    np.add.at(gs, st.tets.ravel(), np.repeat(np.linalg.norm(ge.reshape(T, 12), axis=1), 4))
    wn = np.linalg.norm(st.w, axis=1)
    if len(st.ids):
        np.add.at(gs, st.ids.ravel(), np.repeat(np.abs(st.gfac) * wn, 4))
    gs[fixed] = 0.0
    del ge

    _, _, emap, cmap, diag = oracle.pattern(N, scene["tets"], scene["pt"], scene["ee"])
    bs = np.zeros(len(col))
    np.add.at(bs, emap.ravel(), np.repeat(np.linalg.norm(He.reshape(T, -1), axis=1), emap.shape[1]))
    del He
    if len(st.ids):
        np.add.at(bs, cmap.ravel(), np.repeat(st.hfac * wn ** 2, cmap.shape[1]))
    bs[diag] += np.sqrt(3.0) * st.mass
    rows = np.repeat(np.arange(N), np.diff(row_ptr))
    off = rows != col
    bs[off & (fixed[rows] | fixed[col])] = 0.0
    return gs, bs


def elementwise(g, G, B, Bref, gs, bs):
    """Largest error-to-scale ratios of the gradient per node and of the blocks
    per block; entries with scale 0 must match exactly (reported as inf
    otherwise)."""
    eg = np.linalg.norm(g - G, axis=1)
    eb = np.linalg.norm((B - Bref).reshape(len(B), -1), axis=1)
    with np.errstate(divide="ignore", invalid="ignore"):
        rg = np.where(gs > 0, eg / np.where(gs > 0, gs, 1.0), np.where(eg > 0, np.inf, 0.0))
        rb = np.where(bs > 0, eb / np.where(bs > 0, bs, 1.0), np.where(eb > 0, np.inf, 0.0))
    return float(rg.max(initial=0.0)), float(rb.max(initial=0.0)), int(np.argmax(rg)), int(np.argmax(rb))
