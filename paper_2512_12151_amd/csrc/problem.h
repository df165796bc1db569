// Host-side objects of libbfal shared by the C-ABI (api.hip) and the serving
// engine (server.hip).  Internal: nothing here is part of the C-ABI.
#pragma once

#include <cmath>
#include <string>
#include <vector>

#include "common.h"

using bfal::DevBuf;
using bfal::PcgScalars;
using bfal::PcgSystem;

struct bf_context {
  int device = 0;
  int num_cu = 256;   // compute units of the device (grid sizing)
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
};

struct bf_problem {
  bf_context* ctx = nullptr;
  int N = 0, T = 0;
  // mesh (per-mesh setup)
  DevBuf tets, rest, E, nu, rho, fixed, Dminv9, vol, mu, lam, mass, mat;
  bool has_mat = false;   // per-tet material codes present (else all Neo-Hookean)
  int nnzb_e = 0;
  DevBuf erow_ptr, ecol, emap, ecptr, elist, epos, staging;
  // state
  DevBuf x, xh, xt;
  double dt = 0.0;
  bool has_state = false;
  // constraints
  int n_pt = 0, n_ee = 0, n_c = 0;
  DevBuf cids, clam, cgam;
  double kappa = 1.0, delta = 0.0;
  // semi-implicit friction (Appendix A): the contacts captured at x^t, held for
  // the step; pids = constraints then friction contacts (the pattern's stencils)
  int n_f = 0;
  double fric_e = 0.0;             // eps_v h
  DevBuf fids, f64, fx0, fgk, pids;
  DevBuf ftab, cfr, fextra, fpos, fext;   // per step: friction contact <-> constraint with the same stencil
  // per-step buffers
  DevBuf cg, ch, viol_part;   // AL factors per constraint (FP64)
  DevBuf vcnt, vptr, vinc;
  DevBuf ccount, cptr, cand, ucount, row_ptr, col, eslot;
  DevBuf vals, grad, Lf, Linv, bhat, bb_part, lcnt, lptr, lsrc, sbu, sbl, sblk, sblk16, scol, sent;
  DevBuf wplan_ptr, wplan_sl;                  // the SpMV's slice plan of the current step
  DevBuf cslot;                                // merged-pattern slots of each stencil's ten vertex pairs
  std::vector<int> h_sbu, h_sbl, h_wptr, h_wsl;  // host copies for planning (kept for the async upload)
  DevBuf xs, r, pring, q, part, scal, pout, flags, scan_tmp, scratch_int;
  DevBuf xd, rd, zd, fcg, rpart;   // refinement: FP64 solution, residual, inner solution, directions, partials
  DevBuf lin64;                    // FP64 linearization of the constraints, SoA [8][n]
  DevBuf pdir, xtrial, epart;      // subproblem: Newton direction, line-search trial state, partials
  long long cap_nnzb = 0, cap_cand = 0;
  long long nslot_u = 0, nslot_l = 0;   // slots of the sliced storage of the last step
  PcgScalars* host_sc = nullptr;
  // collision queries: the surface (built at the first call), two BVHs, the
  // colliding pairs and the active-set rebuild
  bool surf_ready = false;
  int nF = 0, nE = 0, nV = 0;
  DevBuf stris, sedges, sverts;
  DevBuf xq;
  DevBuf tbox, tkey, tkey2, tchild, tparent, tnode, tarrive;
  DevBuf ebox, ekey, ekey2, echild, eparent, enode, earrive;
  DevBuf bpart, qcount, qpairs[2], qtoc[2], pkey, pkey2, pidx, pidx2, sort_tmp, ctmp;
  DevBuf htable, tvmin, keepn[2], posn[2], keepc, posc, nids, nlam, ngam, mpart;
  DevBuf xstart, xprev, vout;   // time step: x^t, the subproblem's input x_hat, the velocity
  int qcap[2] = {0, 0};
  int qhits[2] = {0, 0};   // colliding pairs of the last collision call (-1: none yet)
  bool collided = false;
  bool stepped = false;
  bool last_breakdown = false;     // the last step's PCG stopped at p^T H p <= 0 (nothing else failed)
  long long nnzb_last = 0;
  hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  std::vector<hipEvent_t> tev;   // SpMV timing events (pairs), created on demand
};

namespace bfal {

inline bf_status fail(bf_context* c, bf_status st, const std::string& msg) {
  if (c) c->err = msg;
  return st;
}

#define HIPCHK(ctx, call)                                                                  \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail((ctx), e_ == hipErrorOutOfMemory ? BF_ERR_OOM : BF_ERR_HIP,              \
                  std::string(#call) + ": " + hipGetErrorString(e_));                      \
  } while (0)

#define ALLOC(ctx, buf, bytes)                                                             \
  do {                                                                                     \
    hipError_t e_ = (buf).ensure(bytes);                                                   \
    if (e_ != hipSuccess)                                                                  \
      return fail((ctx), BF_ERR_OOM, std::string("device allocation of ") +                \
                  std::to_string((size_t)(bytes)) + " bytes failed");                      \
  } while (0)

inline hipMemcpyKind kind_in(int32_t mem) { return mem == BF_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice; }
inline hipMemcpyKind kind_out(int32_t mem) { return mem == BF_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost; }

inline bool finite_all(const double* a, long long n) {
  for (long long i = 0; i < n; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

inline bf_status flags_to_status(bf_context* c, int flags) {
  if (flags & FLAG_BAD_INDEX) return fail(c, BF_ERR_INVALID_ARG, "index out of range or repeated vertex in a tet");
  if (flags & FLAG_BAD_VALUE) return fail(c, BF_ERR_INVALID_ARG, "invalid value (degenerate rest tet, material, lambda or gamma)");
  if (flags & FLAG_DEGENERATE)
    return fail(c, BF_ERR_DEGENERATE_CONSTRAINT, "degenerate constraint: d(x) <= 0, repeated vertex or parallel edge pair");
  if (flags & FLAG_INVERTED) return fail(c, BF_ERR_INVERTED_ELEMENT, "inverted element: det F(x_hat) <= 0");
  if (flags & (FLAG_NOT_SPD | FLAG_BREAKDOWN)) return fail(c, BF_ERR_NOT_SPD, "matrix not SPD (diagonal block or PCG breakdown)");
  return BF_OK;
}

// The PCG system of a problem's current step (its buffers, grids and row ranges).
inline PcgSystem system_of(bf_problem* pb) {
  PcgSystem S;
  S.N = pb->N;
  S.N4 = (pb->N + 3) & ~3;
  S.nslices = div_up(pb->N, kSlice);
  S.sbu = pb->sbu.as<int>();
  S.sbl = pb->sbl.as<int>();
  S.wave_ptr = pb->wplan_ptr.as<int>();
  S.wave_slices = pb->wplan_sl.as<int>();
  S.scol = pb->scol.as<int>();
  S.blk = pb->sblk.p;
  S.sent = pb->sent.as<int2>();
  S.Lf = pb->Lf.as<float>();
  S.x = pb->xs.as<double>();
  S.r = pb->r.as<float>();
  S.P = pb->pring.as<float>();
  S.pstride = 3LL * S.N4;
  S.q = pb->q.as<float>();
  S.part = pb->part.as<double>();
  S.sc = pb->scal.as<PcgScalars>();
  S.spmv_wg0 = 0;
  S.spmv_nwg = pcg_spmv_groups(pb->N, pb->ctx->num_cu);
  S.vec_wg0 = 0;
  S.vec_nwg = pcg_vec_groups(pb->N);
  return S;
}

inline bf_status read_flags(bf_problem* pb, int* out) {
  bf_context* c = pb->ctx;
  HIPCHK(c, hipMemcpyAsync(out, pb->flags.p, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return BF_OK;
}

// Per-mesh setup of a problem object (fresh or reused: buffers grow as needed).
bf_status problem_init(bf_context* c, bf_problem* pb, const bf_mesh_desc* m, int32_t mem);
// Phases (1)-(3) of a Newton step: constraint linearization, merged pattern,
// assembly with DBC and the block-Jacobi factors, sliced storage (and its BF16
// copy when bf16).  Enqueued on the context's stream; after it system_of(pb)
// describes the step's PCG system.  Assembly errors are raised into pb->flags.
bf_status step_assemble(bf_problem* pb, bool bf16);
// Slots of the table matching friction contacts to constraints: a power of two
// at least twice the constraint count (at least 2), so probes always end.
inline unsigned friction_table_capacity(int n_c) {
  unsigned cap = 2;
  while (cap < 2u * (unsigned)n_c) cap <<= 1;
  return cap;
}
// Sets the constraint counts (PT first) and sizes every per-constraint and
// per-step buffer for them; the constraint arrays themselves are the caller's.
bf_status size_constraint_buffers(bf_problem* pb, int n_pt, int n_ee);

}  // namespace bfal
