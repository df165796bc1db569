// Block-Jacobi preconditioned CG (the paper's linear solver: CG with a 3x3
// block-Jacobi preconditioner on the symmetric BSR matrix, Section 5.1), run on
// the symmetrically scaled system H_hat = L^{-1} H L^{-T} (D_v = L_v L_v^T),
// whose diagonal blocks are identities.  In exact arithmetic its iterates are
// those of PCG with z = D^{-1} r on H: p = L^{-T} p_hat, r = L r_hat.
//
// One iteration is two kernels on one stream, with no host round trip:
//   spmv    convergence test on r_k;
//           q = H_hat p_k = p_k + sum over the stored upper blocks of the row
//           (B_rc p_c) + sum over the upper blocks of its column (B_cr^T p_c);
//           p^T q, r^T q and q^T q (FP64).
//   update  alpha = rho_k / p^T q; beta = rho~_{k+1} / rho_k with
//           rho~_{k+1} = |r - alpha q|^2 = rho_k - 2 alpha r^T q + alpha^2 q^T q
//           (known before r is updated, so the direction can be formed in the
//           same pass); r -= alpha q, p_{k+1} = r_{k+1} + beta p_k into the
//           next buffer of a ring; rho_{k+1} = r^T r (FP64, for the next
//           alpha and the convergence test); every check_every iterations
//           also |L r|^2, the unscaled residual norm squared.  The FP64
//           x += alpha_j p_j is applied every kXBatch iterations for the
//           last kXBatch directions at once (the same FMAs in the same
//           order as one per iteration), so x is read and written once per
//           kXBatch iterations; a flush kernel applies the pending ones
//           before anything reads x.
// Every SpMV gather then reads one vector (p) instead of forming r + beta p
// from two.
// The upper blocks are stored once, in slices of 64 rows with one lane per row
// (slot k of all 64 rows contiguous), and read twice per iteration: streamed
// for the upper part, and gathered through per-row references for the lower
// part.  On a structured mesh the rows of a slice have the same stencil, so the
// lower references of slot k point at consecutive slots of the source slice
// and the p gathers of a slot are consecutive nodes: every access of the SpMV
// is a contiguous run per wavefront.  Workgroups are mapped so that each XCD
// holds one contiguous range of them, and a per-step plan (bf_slice_plan)
// gives every XCD one contiguous window of slices, which its wavefronts sweep
// together, and balances their cost; the whole upper matrix of the large workload (~150 MB) fits
// the 256 MB Infinity Cache.
//
// Residual replacement (reliable updating): x is kept in FP64, and when the
// recursive residual has fallen 100x since the last replacement, or claims
// convergence, the SpMV stops the system with done = 4 and the host replaces
// r by b - H x formed in FP64 from the stored FP32 blocks and re-forms the
// direction from it, p_k = r_k + (rho_k / rho_{k-1}) p_{k-1}; iteration then
// resumes with the usual recurrences (convergence is accepted only on a
// replaced residual).  Without it, thousands of FP32 iterations let the
// recursive residual drift far below the true one on stiff contact systems.
// The requests depend only on the iteration's values, so a system stops at the
// same iterations alone and in a batch.
//
// Grid-wide sums: every workgroup writes one FP64 partial per quantity, and
// every workgroup of the *next* kernel re-sums all partials in the same fixed
// order, so every workgroup derives bit-identical scalars without any device
// fence or atomic (kernel boundaries make the partials visible).  Scalars the
// host polls are written by workgroup 0 of a system only, into fields that no
// workgroup of the same kernel reads: the SpMV writes `done` and `ks` and reads
// `iter` and `brk`; the update kernel writes `iter` and `brk` and reads `done`
// and `ks`.  Once a system has converged its SpMV workgroups re-derive that
// from the unchanged partials and return, and its update workgroups see
// `done`; so the host enqueues iterations in batches and polls between them.
//
// The same kernels serve a batch of independent systems: each workgroup looks
// up its system in a table, so a batch is a block-diagonal system whose
// scalars (alpha, beta, convergence) are kept per system.
#include <hip/hip_ext.h>

#include "common.h"

namespace bfal {

namespace {

constexpr int kSpmvBlock = 256;                    // threads per SpMV workgroup (4 slices)
constexpr int kSlicesPerGroup = kSpmvBlock / kSlice;
static_assert(kSlicesPerGroup == kSpmvWaves, "the slice plan's parts are the SpMV's wavefronts");
constexpr int kVecBlock = 256;                     // threads per update workgroup (4 nodes per thread)

// Sum of v over a workgroup of NT threads, returned to every thread (fixed shuffle/LDS order).
template <int NT>
__device__ inline double block_sum_all(double v) {
  __shared__ double red[NT / kWave];
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < NT / kWave; ++w) s += red[w];
  return s;
}

// Three sums over a workgroup in one LDS round; the results are valid in thread 0.
template <int NT>
__device__ inline void block_sum3(double& a, double& b, double& c) {
  __shared__ double red[3][NT / kWave];
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    a += __shfl_xor(a, off, kWave);
    b += __shfl_xor(b, off, kWave);
    c += __shfl_xor(c, off, kWave);
  }
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) {
    red[0][threadIdx.x / kWave] = a;
    red[1][threadIdx.x / kWave] = b;
    red[2][threadIdx.x / kWave] = c;
  }
  __syncthreads();
  a = b = c = 0.0;
#pragma unroll
  for (int w = 0; w < NT / kWave; ++w) {
    a += red[0][w];
    b += red[1][w];
    c += red[2][w];
  }
}

template <int NT>
__device__ inline double block_max_all(double v) {
  __shared__ double red[NT / kWave];
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, kWave));
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < NT / kWave; ++w) s = fmax(s, red[w]);
  return s;
}

// This thread's share of a partials array of n <= kMaxSpmvParts entries:
// a[t] + a[t + NT] + ... summed in that order, with every load issued before
// the first add (the partials come from other XCDs through the Infinity
// Cache; a dependent chain would wait one round trip per element).
template <int NT>
__device__ __forceinline__ double thread_parts(const double* __restrict__ a, int n) {
  constexpr int kPer = (kMaxSpmvParts + NT - 1) / NT;
  double v[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int k = threadIdx.x + u * NT;
    v[u] = k < n ? a[k] : 0.0;
  }
  double s = v[0];
#pragma unroll
  for (int u = 1; u < kPer; ++u) s += v[u];
  return s;
}

// Three fixed-order sums of part arrays (lengths n0, n1, n2; n = 0 gives 0) in
// one pass: all loads issued together and one LDS round, so a kernel's
// preamble waits for one memory round trip.
template <int NT>
__device__ inline void sum_parts3(const double* __restrict__ a, int na, const double* __restrict__ b, int nb,
                                  const double* __restrict__ c, int nc, double& sa, double& sb, double& sc) {
  __shared__ double red[3][NT / kWave];
  double va = thread_parts<NT>(a, na), vb = thread_parts<NT>(b, nb), vc = thread_parts<NT>(c, nc);
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    va += __shfl_xor(va, off, kWave);
    vb += __shfl_xor(vb, off, kWave);
    vc += __shfl_xor(vc, off, kWave);
  }
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) {
    red[0][threadIdx.x / kWave] = va;
    red[1][threadIdx.x / kWave] = vb;
    red[2][threadIdx.x / kWave] = vc;
  }
  __syncthreads();
  sa = sb = sc = 0.0;
#pragma unroll
  for (int w = 0; w < NT / kWave; ++w) {
    sa += red[0][w];
    sb += red[1][w];
    sc += red[2][w];
  }
}

// Four fixed-order sums in one pass (as sum_parts3).
template <int NT>
__device__ inline void sum_parts4(const double* __restrict__ a, int na, const double* __restrict__ b, int nb,
                                  const double* __restrict__ c, int nc, const double* __restrict__ d, int nd,
                                  double& sa, double& sb, double& sc, double& sd) {
  __shared__ double red[4][NT / kWave];
  double v[4] = {thread_parts<NT>(a, na), thread_parts<NT>(b, nb), thread_parts<NT>(c, nc), thread_parts<NT>(d, nd)};
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1)
#pragma unroll
    for (int m = 0; m < 4; ++m) v[m] += __shfl_xor(v[m], off, kWave);
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0)
#pragma unroll
    for (int m = 0; m < 4; ++m) red[m][threadIdx.x / kWave] = v[m];
  __syncthreads();
  double t[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int w = 0; w < NT / kWave; ++w)
#pragma unroll
    for (int m = 0; m < 4; ++m) t[m] += red[m][w];
  sa = t[0];
  sb = t[1];
  sc = t[2];
  sd = t[3];
}

// Fixed-order sum of part[0..n) by the whole workgroup (same value in every workgroup).
template <int NT>
__device__ inline double sum_parts(const double* __restrict__ part, int n) {
  double s = 0.0;
  for (int k = threadIdx.x; k < n; k += NT) s += part[k];
  return block_sum_all<NT>(s);
}

// Dispatch ids go round-robin over the 8 XCDs: give each XCD one contiguous
// range of logical workgroups.
__device__ inline int xcd_block(int b, int nb) { return (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b; }

__device__ inline void load_block(const float* __restrict__ u, int j, float b[9]) {
  const float* s = u + 9LL * j;
#pragma unroll
  for (int m = 0; m < 9; ++m) b[m] = s[m];
}

// BF16 block: 10 half-words in 5 words, element 2i in the low half of word i.
__device__ inline void load_block(const uint32_t* __restrict__ u, int j, float b[9]) {
  const uint32_t* s = u + 5LL * j;
  uint32_t w[5];
#pragma unroll
  for (int m = 0; m < 5; ++m) w[m] = s[m];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    b[2 * m] = __uint_as_float(w[m] << 16);
    b[2 * m + 1] = __uint_as_float(w[m] & 0xffff0000u);
  }
  b[8] = __uint_as_float(w[4] << 16);
}

// Vector entries of p_k at node c (AoS [N4][3]: one 12-byte load per node).
struct PView {
  const float* __restrict__ p;
  __device__ inline void at(int c, float& p0, float& p1, float& p2) const {
    const float* pc = p + 3LL * c;
    p0 = pc[0];
    p1 = pc[1];
    p2 = pc[2];
  }
};

// Index loads of one step of a row's pairs: upper slot columns from scol,
// lower block slots and source rows from sent.
__device__ __forceinline__ void load_step_indices(const int* __restrict__ scol, const int2* __restrict__ sent,
                                                  int ubase, int lbase, int uc[kPairs], int lb[kPairs],
                                                  int lc[kPairs]) {
#pragma unroll
  for (int u = 0; u < kPairs; ++u) {
    uc[u] = scol[ubase + u * kSlice];
    const int2 t = sent[lbase + u * kSlice];
    lb[u] = t.x;
    lc[u] = t.y;
  }
}

// One step of a row's pairs (upper slot k + u: B p_c with the column from
// scol; lower slot k + u: B^T p_r with block and source row from sent), with
// all its loads issued before any is used.  The step's indices arrive loaded
// (uc, lb, lc); the next step's are loaded before this step's products (a
// scheduling barrier keeps them there), from the next slice's first step
// (bases nub, nlb) after the row's last step.  A step may run past the row's
// widths: those slots are still read (the slot arrays are padded, so every
// index read is in range) but not added, which keeps the step free of
// branches.
template <class BT>
__device__ __forceinline__ void pair_step(int k, int wu, int wl, int w, int ubase, int lbase, int nub, int nlb,
                                          const int* __restrict__ scol, const int2* __restrict__ sent,
                                          const BT* __restrict__ blk, const PView& pv, int uc[kPairs],
                                          int lb[kPairs], int lc[kPairs], float& a0, float& a1, float& a2) {
  float bu[kPairs][9], pu[kPairs][3], bl[kPairs][9], pl[kPairs][3];
#pragma unroll
  for (int u = 0; u < kPairs; ++u) {
    load_block(blk, ubase + (k + u) * kSlice, bu[u]);
    pv.at(uc[u], pu[u][0], pu[u][1], pu[u][2]);
    load_block(blk, lb[u], bl[u]);
    pv.at(lc[u], pl[u][0], pl[u][1], pl[u][2]);
  }
  const bool more = k + kPairs < w;
  load_step_indices(scol, sent, more ? ubase + (k + kPairs) * kSlice : nub, more ? lbase + (k + kPairs) * kSlice : nlb,
                    uc, lb, lc);
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int u = 0; u < kPairs; ++u) {
    const bool vu = k + u < wu, vl = k + u < wl;
    const float y0 = bu[u][0] * pu[u][0] + bu[u][1] * pu[u][1] + bu[u][2] * pu[u][2];
    const float y1 = bu[u][3] * pu[u][0] + bu[u][4] * pu[u][1] + bu[u][5] * pu[u][2];
    const float y2 = bu[u][6] * pu[u][0] + bu[u][7] * pu[u][1] + bu[u][8] * pu[u][2];
    a0 += vu ? y0 : 0.f;
    a1 += vu ? y1 : 0.f;
    a2 += vu ? y2 : 0.f;
    const float z0 = bl[u][0] * pl[u][0] + bl[u][3] * pl[u][1] + bl[u][6] * pl[u][2];
    const float z1 = bl[u][1] * pl[u][0] + bl[u][4] * pl[u][1] + bl[u][7] * pl[u][2];
    const float z2 = bl[u][2] * pl[u][0] + bl[u][5] * pl[u][1] + bl[u][8] * pl[u][2];
    a0 += vl ? z0 : 0.f;
    a1 += vl ? z1 : 0.f;
    a2 += vl ? z2 : 0.f;
  }
}

// A wavefront's place in its slice list (bf_slice_plan): its range [j0, j1),
// the current slice and the next two, the slot offsets of the current and the
// next slice, and the indices of the current slice's first step.
struct SliceCursor {
  int j0, j1, sl, sl1, sl2, bu, eu, bl, el, nbu, neu, nbl, nel;
  int uc[kPairs], lb[kPairs], lc[kPairs];
};

// Start of SpMV k, in one pass of loads: the solver scalars and the partials
// of r^T r and |L r|^2 (which decide whether the system goes on) are loaded
// together with the wavefront's first slices, their offsets and first
// indices, which do not depend on the iteration.  Returns false when the
// system is finished (converged, capped, broken down, or a residual
// replacement is due) and the workgroup must return.  Called by the whole
// workgroup.
__device__ inline bool spmv_begin(const PcgSystem& S, int lb, bool leader, int& k, SliceCursor& c) {
  const int wave = threadIdx.x / kSlice, lane = threadIdx.x % kSlice;
  PcgScalars* sc = S.sc;
  const int every = sc->check_every, brk = sc->brk;
  k = sc->iter;
  const int part = lb * kSlicesPerGroup + wave;
  c.j0 = S.wave_ptr[part];
  c.j1 = S.wave_ptr[part + 1];
  // r^T r and |L r|^2 partials (the latter used on check iterations only);
  // every load is issued (indices past the count re-read the last entry and
  // are not added), so later waits count the loads in order
  constexpr int kPer = (kMaxVecParts + kSpmvBlock - 1) / kSpmvBlock;
  const int nv = S.vec_nwg;
  double va[kPer], vb[kPer];
  {
    const double* pa = S.part + kPartRR + (k & 1) * kMaxVecParts;
    const double* pb = S.part + kPartRT;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int i = min((int)threadIdx.x + u * kSpmvBlock, nv - 1);
      va[u] = pa[i];
      vb[u] = pb[i];
    }
  }
  // an empty range reads slice 0 and is not walked
  const int jf = c.j0 < c.j1 ? c.j0 : 0, jl = c.j0 < c.j1 ? c.j1 - 1 : 0;
  c.sl = S.wave_slices[jf];
  c.sl1 = S.wave_slices[min(jf + 1, jl)];
  c.sl2 = S.wave_slices[min(jf + 2, jl)];
  c.bu = S.sbu[c.sl]; c.eu = S.sbu[c.sl + 1]; c.bl = S.sbl[c.sl]; c.el = S.sbl[c.sl + 1];
  c.nbu = S.sbu[c.sl1]; c.neu = S.sbu[c.sl1 + 1]; c.nbl = S.sbl[c.sl1]; c.nel = S.sbl[c.sl1 + 1];
  load_step_indices(S.scol, S.sent, c.bu + lane, c.bl + lane, c.uc, c.lb, c.lc);
  const bool first = (int)threadIdx.x < nv;
  double a = first ? va[0] : 0.0, b = first ? vb[0] : 0.0;
#pragma unroll
  for (int u = 1; u < kPer; ++u) {
    const bool in = (int)threadIdx.x + u * kSpmvBlock < nv;
    a += in ? va[u] : 0.0;
    b += in ? vb[u] : 0.0;
  }
  double unused = 0.0;
  block_sum3<kSpmvBlock>(a, b, unused);
  const bool check = (k > 0) & ((k % every) == 0);
  const double rho = a, rt = check ? b : 0.0;
  if (brk) return false;
  if (k > 0) {
    const bool converged = (check && rt <= sc->tol2 * sc->bb) || rho == 0.0;
    const bool capped = k >= sc->max_iter;
    // residual replacement: to accept convergence (unless this iteration's
    // residual was just replaced) and whenever |L r| fell 10x since the last one
    const bool replace = sc->replace_on && rho != 0.0 &&
                         ((converged && sc->verified != k) || (!converged && check && rt <= 1e-2 * sc->rt_ref));
    if (leader) {
      sc->rho = rho;
      if (check) sc->rr_true = rt;
      if (replace) sc->done = 4;
      else if (converged) sc->done = 1;
      else if (capped) sc->done = 2;
    }
    if (converged || capped || replace) return false;
  }
  if (leader) sc->ks = k;
  return true;
}

// q = H_hat p_k for the slices of the cursor (bf_slice_plan: each XCD sweeps
// one window of slices, balanced in cost across its waves); adds
// this thread's shares of p^T q, r^T q and q^T q.  The slices are pipelined
// so that a change of slice costs no extra memory round trip: the slot
// offsets are loaded two slices ahead and the slice numbers three ahead, a
// slice's own p and r entries are loaded before its first step, and its last
// step loads the next slice's first indices.  Every slice takes at least one
// step.
template <class BT>
__device__ inline void spmv_slices(const PcgSystem& S, int k, SliceCursor& c, double& pq, double& rq, double& qq) {
  const int lane = threadIdx.x % kSlice;
  const PView pv{S.P + (k % kPRing) * S.pstride};
  const BT* __restrict__ blk = static_cast<const BT*>(S.blk);
  const int jl = c.j1 - 1;
  for (int j = c.j0; j < c.j1; ++j) {
    const int sl3 = S.wave_slices[min(j + 3, jl)];
    const int b2u = S.sbu[c.sl2], e2u = S.sbu[c.sl2 + 1], b2l = S.sbl[c.sl2], e2l = S.sbl[c.sl2 + 1];
    const int row = c.sl * kSlice + lane;
    const bool live = row < S.N;
    // read unconditionally (a pad row reads row N - 1 and is not used), so no
    // branch forces a wait on the loads in flight
    const int rowc = live ? row : S.N - 1;
    float s0, s1, s2;
    pv.at(rowc, s0, s1, s2);
    const float* rr = S.r + 3LL * rowc;
    const float r0 = rr[0], r1 = rr[1], r2 = rr[2];
    const int wu = (c.eu - c.bu) / kSlice, wl = (c.el - c.bl) / kSlice, w = wu > wl ? wu : wl;
    float a0 = 0.f, a1 = 0.f, a2 = 0.f;
    pair_step<BT>(0, wu, wl, w, c.bu + lane, c.bl + lane, c.nbu + lane, c.nbl + lane, S.scol, S.sent, blk, pv, c.uc,
                  c.lb, c.lc, a0, a1, a2);
    for (int kk = kPairs; kk < w; kk += kPairs)
      pair_step<BT>(kk, wu, wl, w, c.bu + lane, c.bl + lane, c.nbu + lane, c.nbl + lane, S.scol, S.sent, blk, pv,
                    c.uc, c.lb, c.lc, a0, a1, a2);
    if (live) {
      const float q0 = s0 + a0, q1 = s1 + a1, q2 = s2 + a2;
      S.q[3LL * row] = q0; S.q[3LL * row + 1] = q1; S.q[3LL * row + 2] = q2;
      pq += (double)s0 * q0 + (double)s1 * q1 + (double)s2 * q2;
      rq += (double)r0 * q0 + (double)r1 * q1 + (double)r2 * q2;
      qq += (double)q0 * q0 + (double)q1 * q1 + (double)q2 * q2;
    }
    c.sl = c.sl1; c.sl1 = c.sl2; c.sl2 = sl3;
    c.bu = c.nbu; c.eu = c.neu; c.bl = c.nbl; c.el = c.nel;
    c.nbu = b2u; c.neu = e2u; c.nbl = b2l; c.nel = e2l;
  }
}

template <class BT>
__global__ void __launch_bounds__(kSpmvBlock) k_spmv(PcgSystem S) {
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  int k;
  SliceCursor c;
  if (!spmv_begin(S, lb, lb == 0 && threadIdx.x == 0, k, c)) return;
  double pq = 0.0, rq = 0.0, qq = 0.0;
  spmv_slices<BT>(S, k, c, pq, rq, qq);
  block_sum3<kSpmvBlock>(pq, rq, qq);
  if (threadIdx.x == 0) {
    S.part[kPartPQ + lb] = pq;
    S.part[kPartRQ + lb] = rq;
    S.part[kPartQQ + lb] = qq;
  }
}

template <class BT>
__global__ void __launch_bounds__(kSpmvBlock) k_spmv_batched(const PcgSystem* __restrict__ sys,
                                                              const int* __restrict__ wg_sys) {
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const PcgSystem S = sys[wg_sys[b]];
  const int lb = b - S.spmv_wg0;
  int k;
  SliceCursor c;
  if (!spmv_begin(S, lb, lb == 0 && threadIdx.x == 0, k, c)) return;
  double pq = 0.0, rq = 0.0, qq = 0.0;
  spmv_slices<BT>(S, k, c, pq, rq, qq);
  block_sum3<kSpmvBlock>(pq, rq, qq);
  if (threadIdx.x == 0) {
    S.part[kPartPQ + lb] = pq;
    S.part[kPartRQ + lb] = rq;
    S.part[kPartQQ + lb] = qq;
  }
}

// Operands of one chunk of 4 * kVecBlock nodes for one thread: three float4
// of p, q, r; on flush iterations the matching FP64 x and the pending
// directions p_j, j0 <= j < k (at most kXBatch - 1; the slots of absent ones
// repeat p_k and are not applied); on check iterations the thread's 4 nodes
// of L (SoA [6][N4]).
struct UpdateOperands {
  float4 p[3], q[3], r[3], l[6];
  double2 xa[3], xb[3];
  float4 pj[kXBatch - 1][3];
};

// Where the directions of iteration k live, and which of them x still lacks
// at the update of iteration k: j0 <= j <= k on a flush iteration.
__device__ __forceinline__ const float* dir_of(const PcgSystem& S, int j) { return S.P + (j % kPRing) * S.pstride; }

__device__ __forceinline__ void load_update_operands(const PcgSystem& S, int k, bool flush, int j0, long long ch,
                                                     bool check, UpdateOperands& o) {
  const int t = threadIdx.x;
  const long long n4 = S.N4, nf4 = 3 * n4 / 4;
  const float4* __restrict__ p4 = reinterpret_cast<const float4*>(dir_of(S, k));
  const float4* __restrict__ q4 = reinterpret_cast<const float4*>(S.q);
  const double2* __restrict__ x2 = reinterpret_cast<const double2*>(S.x);
  const float4* __restrict__ r4 = reinterpret_cast<const float4*>(S.r);
  const float4* __restrict__ l4 = reinterpret_cast<const float4*>(S.Lf);
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    const long long f = ch * 3 * kVecBlock + m * kVecBlock + t;
    if (f < nf4) {
      o.p[m] = p4[f];
      o.q[m] = q4[f];
      o.r[m] = r4[f];
    }
  }
  if (flush) {
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      const long long f = ch * 3 * kVecBlock + m * kVecBlock + t;
      if (f < nf4) {
        o.xa[m] = x2[2 * f];
        o.xb[m] = x2[2 * f + 1];
      }
    }
#pragma unroll
    for (int u = 0; u < kXBatch - 1; ++u) {
      const int j = j0 + u < k ? j0 + u : k;
      const float4* __restrict__ pj4 = reinterpret_cast<const float4*>(dir_of(S, j));
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        const long long f = ch * 3 * kVecBlock + m * kVecBlock + t;
        if (f < nf4) o.pj[u][m] = pj4[f];
      }
    }
  }
  const long long v0 = ch * 4 * kVecBlock + 4LL * t;
  if (check && v0 < n4)
#pragma unroll
    for (int m = 0; m < 6; ++m) o.l[m] = l4[(m * n4 + v0) / 4];
}

// x += alpha_j p_j for j0 <= j <= k, in order (flush iterations only).
__device__ __forceinline__ void apply_pending(double2& xa, double2& xb, const float4 p, const UpdateOperands& o, int m,
                                              int j0, int k, const float* alpha_hist, float alpha) {
#pragma unroll
  for (int u = 0; u < kXBatch - 1; ++u) {
    if (j0 + u < k) {
      const double a = alpha_hist[(j0 + u) % kXBatch];
      const float4 pj = o.pj[u][m];
      xa.x = fma(a, (double)pj.x, xa.x); xa.y = fma(a, (double)pj.y, xa.y);
      xb.x = fma(a, (double)pj.z, xb.x); xb.y = fma(a, (double)pj.w, xb.y);
    }
  }
  const double ad = alpha;   // the same alpha as the residual update
  xa.x = fma(ad, (double)p.x, xa.x); xa.y = fma(ad, (double)p.y, xa.y);
  xb.x = fma(ad, (double)p.z, xb.x); xb.y = fma(ad, (double)p.w, xb.y);
}

// r -= alpha q, p_{k+1} = r + beta p (and on flush iterations the pending
// x updates) for one chunk; adds the chunk's r^T r and (on check iterations)
// |L r|^2 shares.  The new residual is staged in LDS (rs) for the per-node
// |L r|^2.
__device__ __forceinline__ void update_chunk(const PcgSystem& S, float4* __restrict__ pn4, long long ch, bool check,
                                             bool flush, int j0, int k, const float* alpha_hist, float alpha,
                                             float beta, const UpdateOperands& o, float4* rs, double& rr, double& rt) {
  const int t = threadIdx.x;
  const long long n4 = S.N4, nf4 = 3 * n4 / 4;
  double2* __restrict__ x2 = reinterpret_cast<double2*>(S.x);
  float4* __restrict__ r4 = reinterpret_cast<float4*>(S.r);
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    const long long f = ch * 3 * kVecBlock + m * kVecBlock + t;
    if (f < nf4) {
      const float4 p = o.p[m], q = o.q[m];
      float4 r = o.r[m];
      if (flush) {
        double2 xa = o.xa[m], xb = o.xb[m];
        apply_pending(xa, xb, p, o, m, j0, k, alpha_hist, alpha);
        x2[2 * f] = xa;
        x2[2 * f + 1] = xb;
      }
      r.x = __fmaf_rn(-alpha, q.x, r.x); r.y = __fmaf_rn(-alpha, q.y, r.y);
      r.z = __fmaf_rn(-alpha, q.z, r.z); r.w = __fmaf_rn(-alpha, q.w, r.w);
      r4[f] = r;
      pn4[f] = make_float4(__fmaf_rn(beta, p.x, r.x), __fmaf_rn(beta, p.y, r.y), __fmaf_rn(beta, p.z, r.z),
                           __fmaf_rn(beta, p.w, r.w));
      rr += (double)r.x * r.x + (double)r.y * r.y + (double)r.z * r.z + (double)r.w * r.w;
      rs[m * kVecBlock + t] = r;
    }
  }
  if (check) {
    __syncthreads();
    const long long v0 = ch * 4 * kVecBlock + 4LL * t;   // this thread's 4 nodes
    if (v0 < n4) {
      const float4 ra = rs[3 * t], rb = rs[3 * t + 1], rc = rs[3 * t + 2];
      const float rv[12] = {ra.x, ra.y, ra.z, ra.w, rb.x, rb.y, rb.z, rb.w, rc.x, rc.y, rc.z, rc.w};
      const float lx[6][4] = {{o.l[0].x, o.l[0].y, o.l[0].z, o.l[0].w}, {o.l[1].x, o.l[1].y, o.l[1].z, o.l[1].w},
                              {o.l[2].x, o.l[2].y, o.l[2].z, o.l[2].w}, {o.l[3].x, o.l[3].y, o.l[3].z, o.l[3].w},
                              {o.l[4].x, o.l[4].y, o.l[4].z, o.l[4].w}, {o.l[5].x, o.l[5].y, o.l[5].z, o.l[5].w}};
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float* r = rv + 3 * v;
        const double t0 = (double)lx[0][v] * r[0];
        const double t1 = (double)lx[1][v] * r[0] + (double)lx[2][v] * r[1];
        const double t2 = (double)lx[3][v] * r[0] + (double)lx[4][v] * r[1] + (double)lx[5][v] * r[2];
        rt += t0 * t0 + t1 * t1 + t2 * t2;
      }
    }
    __syncthreads();
  }
}

// alpha and beta, then r -= alpha q, p_{k+1} = r + beta p (and x on flush iterations) over
// the nodes of workgroup lb of nwg, in chunks of 4 * kVecBlock nodes whose
// three vectors' float4s are contiguous (every load and store is one
// contiguous run per wavefront).  The operands of the workgroup's first chunk
// are loaded before the grid-wide sums, so their latency overlaps the
// reduction (a workgroup usually owns one chunk).
__device__ inline void update_nodes(const PcgSystem& S, int lb) {
  PcgScalars* sc = S.sc;
  // the control words are read together (k, every and xbase are also used
  // after the test of `done`, so their loads stay with it)
  const int done = sc->done, k = sc->ks, every = sc->check_every, xbase = sc->xbase;
  const bool check = ((k + 1) % every) == 0;
  double* part = S.part;
  __shared__ float4 rs[3 * kVecBlock];
  __shared__ float alpha_hist[kXBatch];
  float4* __restrict__ pn4 = reinterpret_cast<float4*>(const_cast<float*>(dir_of(S, k + 1)));
  const long long nchunk = (S.N4 + 4 * kVecBlock - 1) / (4 * kVecBlock);
  // x takes alpha_j p_j, j0 <= j <= k, on every kXBatch-th iteration
  const bool flush = ((k + 1) % kXBatch) == 0;
  const int j0 = max(xbase, k + 1 - kXBatch);
  UpdateOperands o;
  if (!done && lb < nchunk) load_update_operands(S, k, flush, j0, lb, check, o);
  if (done) return;
  const float ah = sc->alpha_hist[threadIdx.x % kXBatch];
  double rho, pq, rq, qq;
  sum_parts4<kVecBlock>(part + kPartRR + (k & 1) * kMaxVecParts, S.vec_nwg, part + kPartPQ, S.spmv_nwg,
                        part + kPartRQ, S.spmv_nwg, part + kPartQQ, S.spmv_nwg, rho, pq, rq, qq);
  const bool leader = lb == 0 && threadIdx.x == 0;
  if (!(pq > 0.0)) {
    if (leader) {
      sc->flags |= FLAG_BREAKDOWN;
      sc->brk = 1;
    }
    return;
  }
  const float alpha = (float)(rho / pq);
  // |r - alpha q|^2 with the alpha the residual update applies; a negative
  // value (rounding, once r ~ 0) restarts the direction
  const double ad = alpha;
  const double rho_next = rho - 2.0 * ad * rq + ad * ad * qq;
  const float beta = rho_next > 0.0 ? (float)(rho_next / rho) : 0.f;
  double rr = 0.0, rt = 0.0;
  if (flush && threadIdx.x < kXBatch) alpha_hist[threadIdx.x] = ah;
  __syncthreads();   // alpha_hist staged
  if (lb < nchunk) update_chunk(S, pn4, lb, check, flush, j0, k, alpha_hist, alpha, beta, o, rs, rr, rt);
  for (long long ch = lb + S.vec_nwg; ch < nchunk; ch += S.vec_nwg) {
    load_update_operands(S, k, flush, j0, ch, check, o);
    update_chunk(S, pn4, ch, check, flush, j0, k, alpha_hist, alpha, beta, o, rs, rr, rt);
  }
  double unused = 0.0;
  block_sum3<kVecBlock>(rr, rt, unused);   // one LDS round for both sums
  if (threadIdx.x == 0) {
    part[kPartRR + ((k + 1) & 1) * kMaxVecParts + lb] = rr;
    part[kPartRT + lb] = rt;
  }
  if (leader) {
    sc->alpha_hist[k % kXBatch] = alpha;
    sc->iter = k + 1;
  }
}

__global__ void __launch_bounds__(kVecBlock) k_update(PcgSystem S) { update_nodes(S, blockIdx.x); }

__global__ void __launch_bounds__(kVecBlock) k_update_batched(const PcgSystem* __restrict__ sys,
                                                             const int* __restrict__ wg_sys) {
  const PcgSystem S = sys[wg_sys[blockIdx.x]];
  update_nodes(S, blockIdx.x - S.vec_wg0);
}

__global__ void __launch_bounds__(kVecBlock)
k_init(int n3, const float* __restrict__ bhat, double* __restrict__ x, float* __restrict__ r, float* __restrict__ p0,
       double* __restrict__ part) {
  double rr = 0.0;
  for (int i = blockIdx.x * kVecBlock + threadIdx.x; i < n3; i += gridDim.x * kVecBlock) {
    const float b = bhat[i];
    x[i] = 0.0;
    r[i] = b;
    p0[i] = b;
    rr += (double)b * b;
  }
  const double s = block_sum_all<kVecBlock>(rr);
  if (threadIdx.x == 0) part[kPartRR + blockIdx.x] = s;   // iteration 0 reads slot 0
}

__global__ void __launch_bounds__(kBlock)
k_init_scalars(const double* __restrict__ bb_part, int nbb, PcgScalars* sc, double tol, int max_iter,
               int check_every, int replace) {
  const double bb = sum_parts<kBlock>(bb_part, nbb);
  if (threadIdx.x == 0) {
    sc->rt_ref = bb;
    sc->verified = -1;
    sc->replace_on = replace;
    sc->bb = bb;
    sc->rr_true = bb;
    sc->rho = 0.0;
    sc->tol2 = tol * tol;
    sc->iter = 0;
    sc->ks = 0;
    sc->max_iter = max_iter;
    sc->check_every = check_every > 0 ? check_every : 1;
    sc->flags = 0;
    sc->brk = 0;
    sc->xbase = 0;
    sc->done = (bb == 0.0) ? 1 : (max_iter <= 0 ? 2 : 0);
  }
}

// p = L^{-T} x in FP64 (x FP32 or FP64, AoS [N4][3]) and the per-workgroup max |p|.
template <class XT>
__global__ void __launch_bounds__(kVecBlock)
k_finish(int N, int N4, const double* __restrict__ Linv, const XT* __restrict__ x, double* __restrict__ pout,
         double* __restrict__ part) {
  double m = 0.0;
  for (int v = blockIdx.x * kVecBlock + threadIdx.x; v < N; v += gridDim.x * kVecBlock) {
    const double* l = Linv + 6LL * v;
    const double x0 = x[3LL * v], x1 = x[3LL * v + 1], x2 = x[3LL * v + 2];
    const double p0 = l[0] * x0 + l[1] * x1 + l[3] * x2;
    const double p1 = l[2] * x1 + l[4] * x2;
    const double p2 = l[5] * x2;
    pout[3LL * v] = p0;
    pout[3LL * v + 1] = p1;
    pout[3LL * v + 2] = p2;
    m = fmax(m, fmax(fabs(p0), fmax(fabs(p1), fabs(p2))));
  }
  const double s = block_max_all<kVecBlock>(m);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// ------------------------------------------------ iterative refinement
// The outer loop of the BF16 mode keeps the solution x_hat in FP64 and forms
// the residual of the FP32-stored system in FP64: r = b_hat - H_hat x_hat,
// with the FP32 blocks widened to FP64 (the same sliced storage and access
// pattern as the SpMV), plus the per-workgroup partials of |L r|^2.
__global__ void __launch_bounds__(kSpmvBlock)
k_residual64(PcgSystem S, const float* __restrict__ bhat, const double* __restrict__ xd, double* __restrict__ rd,
             double* __restrict__ part) {
  // with bhat == nullptr: rd = H_hat xd and no partials
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int wave = threadIdx.x / kSlice, lane = threadIdx.x % kSlice;
  const float* __restrict__ blk = static_cast<const float*>(S.blk);
  double rt = 0.0;
  for (int sl = lb * kSlicesPerGroup + wave; sl < S.nslices; sl += gridDim.x * kSlicesPerGroup) {
    const int bu = S.sbu[sl], wu = (S.sbu[sl + 1] - bu) / kSlice;
    const int bl = S.sbl[sl], wl = (S.sbl[sl + 1] - bl) / kSlice;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int kk = 0; kk < wu; ++kk) {
      const int e = bu + kk * kSlice + lane;
      const int c = S.scol[e];
      float b[9];
      load_block(blk, e, b);
      const double x0 = xd[3LL * c], x1 = xd[3LL * c + 1], x2 = xd[3LL * c + 2];
      a0 += (double)b[0] * x0 + (double)b[1] * x1 + (double)b[2] * x2;
      a1 += (double)b[3] * x0 + (double)b[4] * x1 + (double)b[5] * x2;
      a2 += (double)b[6] * x0 + (double)b[7] * x1 + (double)b[8] * x2;
    }
    for (int kk = 0; kk < wl; ++kk) {
      const int2 t = S.sent[bl + kk * kSlice + lane];
      const int c = t.y;
      float b[9];
      load_block(blk, t.x, b);
      const double x0 = xd[3LL * c], x1 = xd[3LL * c + 1], x2 = xd[3LL * c + 2];
      a0 += (double)b[0] * x0 + (double)b[3] * x1 + (double)b[6] * x2;
      a1 += (double)b[1] * x0 + (double)b[4] * x1 + (double)b[7] * x2;
      a2 += (double)b[2] * x0 + (double)b[5] * x1 + (double)b[8] * x2;
    }
    const int row = sl * kSlice + lane;
    const long long o = 3LL * row;
    if (row < S.N && !bhat) {
      rd[o] = xd[o] + a0;
      rd[o + 1] = xd[o + 1] + a1;
      rd[o + 2] = xd[o + 2] + a2;
    } else if (row < S.N) {
      const double r0 = (double)bhat[o] - (xd[o] + a0);
      const double r1 = (double)bhat[o + 1] - (xd[o + 1] + a1);
      const double r2 = (double)bhat[o + 2] - (xd[o + 2] + a2);
      rd[o] = r0;
      rd[o + 1] = r1;
      rd[o + 2] = r2;
      const float* L = S.Lf + row;   // SoA [6][N4]
      const long long n4 = S.N4;
      const double t0 = (double)L[0] * r0;
      const double t1 = (double)L[n4] * r0 + (double)L[2 * n4] * r1;
      const double t2 = (double)L[3 * n4] * r0 + (double)L[4 * n4] * r1 + (double)L[5 * n4] * r2;
      rt += t0 * t0 + t1 * t1 + t2 * t2;
    }
  }
  const double s = block_sum_all<kSpmvBlock>(rt);
  if (threadIdx.x == 0 && part) part[lb] = s;
}

// Up to kMaxDots FP64 dot products a . b_j in one pass: partials part[j][blockIdx].
constexpr int kMaxDots = 6;
constexpr int kDotGrid = 256;
struct DotArgs {
  const double* b[kMaxDots];
  int nb;
};

__global__ void __launch_bounds__(kVecBlock)
k_dots64(int n3, const double* __restrict__ a, DotArgs B, double* __restrict__ part) {
  double acc[kMaxDots];
#pragma unroll
  for (int j = 0; j < kMaxDots; ++j) acc[j] = 0.0;
  for (int i = blockIdx.x * kVecBlock + threadIdx.x; i < n3; i += gridDim.x * kVecBlock) {
    const double av = a[i];
#pragma unroll
    for (int j = 0; j < kMaxDots; ++j)
      if (j < B.nb) acc[j] += av * B.b[j][i];
  }
#pragma unroll
  for (int j = 0; j < kMaxDots; ++j) {
    if (j >= B.nb) break;
    const double s = block_sum_all<kVecBlock>(acc[j]);
    if (threadIdx.x == 0) part[j * kDotGrid + blockIdx.x] = s;
  }
}

__global__ void __launch_bounds__(kBlock) k_dots_sum(const double* __restrict__ part, int nb, double* out) {
  for (int j = 0; j < nb; ++j) {
    const double s = sum_parts<kBlock>(part + j * kDotGrid, kDotGrid);
    if (threadIdx.x == 0) out[j] = s;
  }
}

// y += alpha x (FP64).
__global__ void __launch_bounds__(kVecBlock)
k_axpy_d(int n3, double alpha, const double* __restrict__ x, double* __restrict__ y) {
  for (int i = blockIdx.x * kVecBlock + threadIdx.x; i < n3; i += gridDim.x * kVecBlock) y[i] += alpha * x[i];
}

// y = x widened from FP32 to FP64.
__global__ void __launch_bounds__(kVecBlock)
k_copy_f2d(int n3, const float* __restrict__ x, double* __restrict__ y) {
  for (int i = blockIdx.x * kVecBlock + threadIdx.x; i < n3; i += gridDim.x * kVecBlock) y[i] = (double)x[i];
}

// Inner solve start: r = (float) r_outer, x = 0, partials of r^T r.
__global__ void __launch_bounds__(kVecBlock)
k_init_from64(int n3, const double* __restrict__ rd, double* __restrict__ x, float* __restrict__ r,
              float* __restrict__ p0, double* __restrict__ part) {
  double rr = 0.0;
  for (int i = blockIdx.x * kVecBlock + threadIdx.x; i < n3; i += gridDim.x * kVecBlock) {
    const float b = (float)rd[i];
    x[i] = 0.0;
    r[i] = b;
    p0[i] = b;
    rr += (double)b * b;
  }
  const double s = block_sum_all<kVecBlock>(rr);
  if (threadIdx.x == 0) part[kPartRR + blockIdx.x] = s;
}

// x += alpha_j p_j for the directions the update kernel has not applied yet
// (j from the last multiple of kXBatch, or xbase, up to iter - 1), in
// order; then xbase = iter.  Runs before anything reads x.
__global__ void __launch_bounds__(kVecBlock) k_flush_x(PcgSystem S) {
  PcgScalars* sc = S.sc;
  const int n = sc->iter;
  const int j0 = max(sc->xbase, n - n % kXBatch);
  const long long n3 = 3LL * S.N4;
  for (long long i = (long long)blockIdx.x * kVecBlock + threadIdx.x; i < n3; i += (long long)gridDim.x * kVecBlock) {
    double x = S.x[i];
    for (int j = j0; j < n; ++j) x = fma((double)sc->alpha_hist[j % kXBatch], (double)dir_of(S, j)[i], x);
    S.x[i] = x;
  }
}

// Marks the flushed directions (after k_flush_x, in a kernel of its own so
// that no workgroup of the flush reads a changed xbase).
__global__ void k_flush_mark(PcgScalars* sc) {
  if (threadIdx.x == 0 && blockIdx.x == 0) sc->xbase = sc->iter;
}

// Residual replacement, second half: r = (float) rd over this workgroup's
// chunk with its r^T r partial, the |L rd|^2 partials of k_residual64 folded
// into workgroup 0's slot, the reference and the replaced iteration recorded,
// and the system released (done = 0).
__global__ void __launch_bounds__(kVecBlock)
k_replace_fold(PcgSystem S, const double* __restrict__ rd, const double* __restrict__ rpart, int nparts) {
  PcgScalars* sc = S.sc;
  const int k = sc->iter;
  const int lb = blockIdx.x;
  const double rt = sum_parts<kVecBlock>(rpart, nparts);
  const long long n3 = 3LL * S.N4;
  const long long chunk = 12LL * kVecBlock;   // 4 * kVecBlock nodes, as in the update kernel
  double rr = 0.0;
  for (long long c0 = (long long)lb * chunk; c0 < n3; c0 += (long long)gridDim.x * chunk)
    for (long long i = c0 + threadIdx.x; i < c0 + chunk && i < n3; i += kVecBlock) {
      const float r = (float)rd[i];
      S.r[i] = r;
      rr += (double)r * r;
    }
  const double srr = block_sum_all<kVecBlock>(rr);
  if (threadIdx.x == 0) {
    S.part[kPartRR + (k & 1) * kMaxVecParts + lb] = srr;
    S.part[kPartRT + lb] = lb == 0 ? rt : 0.0;
  }
  if (lb == 0 && threadIdx.x == 0) {
    sc->rt_ref = rt;
    sc->rr_true = rt;
    sc->verified = k;
    sc->done = 0;
  }
}

// After a residual replacement at iteration k: p_k = r_k + (rho_k / rho_{k-1})
// p_{k-1} from the replaced residual (p_{k-1} is still in the other buffer).
__global__ void __launch_bounds__(kVecBlock) k_replace_dir(PcgSystem S) {
  const int k = S.sc->iter;
  double rho, rho_old, unused;
  sum_parts3<kVecBlock>(S.part + kPartRR + (k & 1) * kMaxVecParts, S.vec_nwg,
                        S.part + kPartRR + ((k + 1) & 1) * kMaxVecParts, S.vec_nwg, S.part, 0, rho, rho_old, unused);
  const float beta = rho_old > 0.0 ? (float)(rho / rho_old) : 0.f;
  float* __restrict__ pk = const_cast<float*>(dir_of(S, k));
  const float* __restrict__ pold = dir_of(S, k - 1);
  const long long n3 = 3LL * S.N4;
  for (long long i = (long long)blockIdx.x * kVecBlock + threadIdx.x; i < n3; i += (long long)gridDim.x * kVecBlock)
    pk[i] = __fmaf_rn(beta, pold[i], S.r[i]);
}

// x_outer += d (FP64).
__global__ void __launch_bounds__(kVecBlock)
k_axpy64(int n3, const double* __restrict__ d, double* __restrict__ xd) {
  for (int i = blockIdx.x * kVecBlock + threadIdx.x; i < n3; i += gridDim.x * kVecBlock) xd[i] += d[i];
}

__global__ void __launch_bounds__(kBlock) k_sum_to(const double* __restrict__ part, int n, double* out) {
  const double s = sum_parts<kBlock>(part, n);
  if (threadIdx.x == 0) *out = s;
}

__global__ void __launch_bounds__(kBlock)
k_finish_scalars(const double* __restrict__ part, int n, const double* __restrict__ viol_part, int nviol,
                 PcgScalars* sc) {
  double m = 0.0, vm = 0.0;
  for (int k = threadIdx.x; k < n; k += kBlock) m = fmax(m, part[k]);
  for (int k = threadIdx.x; k < nviol; k += kBlock) vm = fmax(vm, viol_part[k]);
  m = block_max_all<kBlock>(m);
  vm = block_max_all<kBlock>(vm);
  if (threadIdx.x == 0) {
    sc->stat_pinf = m;
    sc->stat_viol = vm;
  }
}

}  // namespace

// At most one SpMV workgroup per compute unit: the SpMV is bound by what one
// CU can keep in flight, so a CU holding two workgroups would take twice as
// long as the others (measured on the large workload: 1576 workgroups, 6 or 7
// per CU, 44.5 us; 256, one per CU with 6 or 7 slices per wave, 42.6 us; 264
// or 320, 54 and 65 us).  Each wavefront then walks the slices the plan gives
// it, one window per XCD swept by all its wavefronts together, so the
// lower-half reads of a block mostly follow its upper-half read closely and
// on the same XCD.
int pcg_spmv_groups(int N, int num_cu) {
  const int nslices = div_up(N, kSlice);
  int g = div_up(nslices, kSlicesPerGroup);
  const int cap = num_cu >= 8 ? num_cu / 8 * 8 : 8;
  if (g > cap) g = cap;
  if (g > kMaxSpmvParts) g = kMaxSpmvParts;
  return ((g + 7) / 8) * 8;
}

int pcg_vec_groups(int N) {
  const int ng = ((N + 3) & ~3) / 4;   // chunks of 4 * kVecBlock nodes
  int g = div_up(ng, kVecBlock);
  if (g > kMaxVecParts) g = kMaxVecParts;
  return g < 1 ? 1 : g;
}

void launch_pcg_init(const PcgSystem& S, const float* bhat, const double* bb_part, int nbb, double tol, int max_iter,
                     int check_every, bool replace, hipStream_t s) {
  hipLaunchKernelGGL(k_init, dim3(S.vec_nwg), dim3(kVecBlock), 0, s, 3 * S.N4, bhat, S.x, S.r, S.P, S.part);
  hipLaunchKernelGGL(k_init_scalars, dim3(1), dim3(kBlock), 0, s, bb_part, nbb, S.sc, tol, max_iter, check_every,
                     replace ? 1 : 0);
}

void launch_pcg_flush(const PcgSystem& S, hipStream_t s) {
  hipLaunchKernelGGL(k_flush_x, dim3(S.vec_nwg), dim3(kVecBlock), 0, s, S);
  hipLaunchKernelGGL(k_flush_mark, dim3(1), dim3(64), 0, s, S.sc);
}

void launch_pcg_replace(const PcgSystem& S, const float* bhat, double* rd, double* rpart, hipStream_t s) {
  launch_pcg_flush(S, s);
  hipLaunchKernelGGL(k_residual64, dim3(S.spmv_nwg), dim3(kSpmvBlock), 0, s, S, bhat, (const double*)S.x, rd, rpart);
  hipLaunchKernelGGL(k_replace_fold, dim3(S.vec_nwg), dim3(kVecBlock), 0, s, S, (const double*)rd,
                     (const double*)rpart, S.spmv_nwg);
  hipLaunchKernelGGL(k_replace_dir, dim3(S.vec_nwg), dim3(kVecBlock), 0, s, S);
}

void launch_pcg_iteration(const PcgSystem& S, bool bf16, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
  // with events: the command processor stamps them around the SpMV dispatch itself
  if (t0 && t1) {
    if (bf16)
      hipExtLaunchKernelGGL(k_spmv<uint32_t>, dim3(S.spmv_nwg), dim3(kSpmvBlock), 0, s, t0, t1, 0, S);
    else
      hipExtLaunchKernelGGL(k_spmv<float>, dim3(S.spmv_nwg), dim3(kSpmvBlock), 0, s, t0, t1, 0, S);
  } else if (bf16) {
    hipLaunchKernelGGL(k_spmv<uint32_t>, dim3(S.spmv_nwg), dim3(kSpmvBlock), 0, s, S);
  } else {
    hipLaunchKernelGGL(k_spmv<float>, dim3(S.spmv_nwg), dim3(kSpmvBlock), 0, s, S);
  }
  hipLaunchKernelGGL(k_update, dim3(S.vec_nwg), dim3(kVecBlock), 0, s, S);
}

void launch_pcg_iteration_batched(const PcgSystem* sys, const int* wg_sys_spmv, int nwg_spmv, const int* wg_sys_vec,
                                  int nwg_vec, bool bf16, hipStream_t s) {
  if (bf16)
    hipLaunchKernelGGL(k_spmv_batched<uint32_t>, dim3(nwg_spmv), dim3(kSpmvBlock), 0, s, sys, wg_sys_spmv);
  else
    hipLaunchKernelGGL(k_spmv_batched<float>, dim3(nwg_spmv), dim3(kSpmvBlock), 0, s, sys, wg_sys_spmv);
  hipLaunchKernelGGL(k_update_batched, dim3(nwg_vec), dim3(kVecBlock), 0, s, sys, wg_sys_vec);
}

void launch_pcg_finish(const PcgSystem& S, const double* Linv, double* pout, const double* viol_part, int nviol,
                       hipStream_t s) {
  const int g = pcg_vec_groups(S.N);
  launch_pcg_flush(S, s);
  // the max |p| partials reuse the p^T q slots, which the solve no longer needs
  double* part = S.part + kPartPQ;
  hipLaunchKernelGGL(k_finish<double>, dim3(g), dim3(kVecBlock), 0, s, S.N, S.N4, Linv, (const double*)S.x, pout,
                     part);
  hipLaunchKernelGGL(k_finish_scalars, dim3(1), dim3(kBlock), 0, s, (const double*)part, g, viol_part, nviol, S.sc);
}

void launch_pcg_init_from64(const PcgSystem& S, const double* rd, const double* rpart, int nparts, double tol,
                            int max_iter, int check_every, hipStream_t s) {
  hipLaunchKernelGGL(k_init_from64, dim3(S.vec_nwg), dim3(kVecBlock), 0, s, 3 * S.N4, rd, S.x, S.r, S.P, S.part);
  hipLaunchKernelGGL(k_init_scalars, dim3(1), dim3(kBlock), 0, s, rpart, nparts, S.sc, tol, max_iter, check_every,
                     0);
}

void launch_residual64(const PcgSystem& S, const float* bhat, const double* xd, double* rd, double* rpart,
                       double* rsum, hipStream_t s) {
  hipLaunchKernelGGL(k_residual64, dim3(S.spmv_nwg), dim3(kSpmvBlock), 0, s, S, bhat, xd, rd, rpart);
  hipLaunchKernelGGL(k_sum_to, dim3(1), dim3(kBlock), 0, s, (const double*)rpart, S.spmv_nwg, rsum);
}

void launch_sum_to(const double* part, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_to, dim3(1), dim3(kBlock), 0, s, part, n, out);
}

void launch_apply64(const PcgSystem& S, const double* xd, double* yd, hipStream_t s) {
  hipLaunchKernelGGL(k_residual64, dim3(S.spmv_nwg), dim3(kSpmvBlock), 0, s, S, (const float*)nullptr, xd, yd,
                     (double*)nullptr);
}

void launch_dots64(int n3, const double* a, const double* const* b, int nb, double* part, double* out,
                   hipStream_t s) {
  DotArgs B{};
  for (int j = 0; j < nb && j < kMaxDots; ++j) B.b[j] = b[j];
  B.nb = nb < kMaxDots ? nb : kMaxDots;
  hipLaunchKernelGGL(k_dots64, dim3(kDotGrid), dim3(kVecBlock), 0, s, n3, a, B, part);
  hipLaunchKernelGGL(k_dots_sum, dim3(1), dim3(kBlock), 0, s, (const double*)part, B.nb, out);
}

void launch_axpy_d(int n3, double alpha, const double* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy_d, dim3(div_up(n3, kVecBlock) < 1024 ? div_up(n3, kVecBlock) : 1024), dim3(kVecBlock), 0,
                     s, n3, alpha, x, y);
}

void launch_copy_f2d(int n3, const float* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_f2d, dim3(div_up(n3, kVecBlock) < 1024 ? div_up(n3, kVecBlock) : 1024), dim3(kVecBlock),
                     0, s, n3, x, y);
}

void launch_axpy64(const PcgSystem& S, double* xd, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy64, dim3(S.vec_nwg), dim3(kVecBlock), 0, s, 3 * S.N4, (const double*)S.x, xd);
}

void launch_pcg_finish64(const PcgSystem& S, const double* Linv, const double* xd, double* pout,
                         const double* viol_part, int nviol, hipStream_t s) {
  const int g = pcg_vec_groups(S.N);
  double* part = S.part + kPartPQ;
  hipLaunchKernelGGL(k_finish<double>, dim3(g), dim3(kVecBlock), 0, s, S.N, S.N4, Linv, xd, pout, part);
  hipLaunchKernelGGL(k_finish_scalars, dim3(1), dim3(kBlock), 0, s, (const double*)part, g, viol_part, nviol, S.sc);
}

}  // namespace bfal
