// Per-step constraint kernels.
//  - Linearization (Algorithm 2, before the Newton loop; Section 4.2): for every
//    PT / EE pair, the closest points of the closed primitives at the
//    intersection-free state x give d_i(x), the unit normal n and the weights w,
//    so grad d_i = (w_0 n, w_1 n, w_2 n, w_3 n).  Computed in FP64 from the FP64
//    state (distances of ~1e-3 between coordinates of ~1 would lose 3-4 digits
//    in FP32), then stored in FP32.
//  - The AL factors of the contact loop of Algorithm 2: s_i = max(0, c_i -
//    lambda_i/kappa), gradient factor kappa gamma (c - lambda/kappa - s) and
//    Hessian factor kappa gamma (kept also when s_i > 0).
//  - The merged upper 3x3-block pattern: static elastic rows united with the
//    vertex pairs of the constraints, sorted and unique per row.
#include "common.h"

namespace bfal {

namespace {

struct d3 { double x, y, z; };
__device__ inline d3 ld3(const double* p, int v) {
  const long long o = 3LL * v;
  return {p[o], p[o + 1], p[o + 2]};
}
__device__ inline d3 sub(d3 a, d3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline d3 add(d3 a, d3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ inline d3 mul(d3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
__device__ inline double dot(d3 a, d3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline d3 cross(d3 a, d3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
__device__ inline double clamp01(double t) { return t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t); }

// Parameter of the point of segment [u, u+e] closest to p, clamped to [0, 1].
__device__ inline double seg_param(d3 p, d3 u, d3 e) { return clamp01(dot(sub(p, u), e) / dot(e, e)); }

__device__ inline int vtx(const int4& t, int a) { return a == 0 ? t.x : a == 1 ? t.y : a == 2 ? t.z : t.w; }

// Closest points of a PT pair (point X0, triangle X1 X2 X3: interior projection
// if inside, else the best edge point) or an EE pair (segments X0 X1 and
// X2 X3) at x: diff = (point of the first primitive) - (point of the second)
// = sum_a w_a X_a.  Returns true for a degenerate pair (sliver triangle,
// near-parallel edges) whose gradient is not unique.
__device__ inline bool closest_pair(const int4 t, bool is_pt, const double* __restrict__ x, d3& diff, double w[4]) {
  const d3 X0 = ld3(x, t.x), X1 = ld3(x, t.y), X2 = ld3(x, t.z), X3 = ld3(x, t.w);
  double w0, w1, w2, w3;
  bool degenerate = false;
  if (is_pt) {
    // point X0 against triangle (X1, X2, X3): interior projection if inside, else best edge point
    const d3 e1 = sub(X2, X1), e2 = sub(X3, X1), r = sub(X0, X1);
    const double a11 = dot(e1, e1), a12 = dot(e1, e2), a22 = dot(e2, e2);
    const double r1 = dot(e1, r), r2 = dot(e2, r);
    const double det = a11 * a22 - a12 * a12;
    degenerate = !(det > 1e-12 * a11 * a22);
    double best = INFINITY, b0 = 1.0, b1 = 0.0, b2 = 0.0;
    if (!degenerate) {
      const double u = (a22 * r1 - a12 * r2) / det, v = (a11 * r2 - a12 * r1) / det;
      if (u >= 0.0 && v >= 0.0 && u + v <= 1.0) {
        const d3 q = add(X1, add(mul(e1, u), mul(e2, v)));
        const d3 dd = sub(X0, q);
        best = sqrt(dot(dd, dd));
        b0 = 1.0 - u - v; b1 = u; b2 = v;
      }
    }
    const d3 T[3] = {X1, X2, X3};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int ia = k, ib = (k + 1) % 3;
      const double s = seg_param(X0, T[ia], sub(T[ib], T[ia]));
      const d3 q = add(T[ia], mul(sub(T[ib], T[ia]), s));
      const d3 dd = sub(X0, q);
      const double dist = sqrt(dot(dd, dd));
      if (dist < best) {
        best = dist;
        double bb[3] = {0.0, 0.0, 0.0};
        bb[ia] = 1.0 - s; bb[ib] = s;
        b0 = bb[0]; b1 = bb[1]; b2 = bb[2];
      }
    }
    const d3 q = add(add(mul(X1, b0), mul(X2, b1)), mul(X3, b2));
    diff = sub(X0, q);
    w0 = 1.0; w1 = -b0; w2 = -b1; w3 = -b2;
  } else {
    // segments X0 + s (X1 - X0) and X2 + t (X3 - X2)
    const d3 ea = sub(X1, X0), eb = sub(X3, X2), r = sub(X0, X2);
    const double aa = dot(ea, ea), bb = dot(eb, eb), ab = dot(ea, eb);
    const double ar = dot(ea, r), br = dot(eb, r);
    const d3 cr = cross(ea, eb);
    degenerate = dot(cr, cr) < 1e-8 * aa * bb;   // (near-)parallel pair: gradient not unique
    const double det = aa * bb - ab * ab;
    double best = INFINITY, sb = 0.0, tb = 0.0;
    if (!degenerate && det > 0.0) {
      const double s = (-ar * bb + ab * br) / det, tt = (aa * br - ab * ar) / det;
      if (s >= 0.0 && s <= 1.0 && tt >= 0.0 && tt <= 1.0) {
        const d3 dd = sub(add(X0, mul(ea, s)), add(X2, mul(eb, tt)));
        best = sqrt(dot(dd, dd));
        sb = s; tb = tt;
      }
    }
    const double cs[4] = {0.0, 1.0, seg_param(X2, X0, ea), seg_param(X3, X0, ea)};
    const double ct[4] = {seg_param(X0, X2, eb), seg_param(X1, X2, eb), 0.0, 1.0};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const d3 dd = sub(add(X0, mul(ea, cs[k])), add(X2, mul(eb, ct[k])));
      const double dist = sqrt(dot(dd, dd));
      if (dist < best) { best = dist; sb = cs[k]; tb = ct[k]; }
    }
    diff = sub(add(X0, mul(ea, sb)), add(X2, mul(eb, tb)));
    w0 = 1.0 - sb; w1 = sb; w2 = -(1.0 - tb); w3 = -tb;
  }
  w[0] = w0; w[1] = w1; w[2] = w2; w[3] = w3;
  return degenerate;
}

__global__ void k_check_constraints(const int4* __restrict__ ids, int n_c, int N, const double* __restrict__ lam,
                                    const double* __restrict__ gam, int* flags) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_c) return;
  const int4 t = ids[i];
  bool bad = t.x < 0 || t.y < 0 || t.z < 0 || t.w < 0 || t.x >= N || t.y >= N || t.z >= N || t.w >= N;
  if (bad) { atomicOr(flags, FLAG_BAD_INDEX); return; }
  if (t.x == t.y || t.x == t.z || t.x == t.w || t.y == t.z || t.y == t.w || t.z == t.w)
    atomicOr(flags, FLAG_DEGENERATE);
  const double l = lam[i], g = gam[i];
  if (!(l >= 0.0 && l < INFINITY) || !(g > 0.0 && g <= 1.0)) atomicOr(flags, FLAG_BAD_VALUE);
}

__global__ void __launch_bounds__(kBlock)
k_contact_lin(const int4* __restrict__ ids, int n_pt, int n_c, const double* __restrict__ x,
              const double* __restrict__ xh, const double* __restrict__ lam, const double* __restrict__ gam,
              double kappa, double delta, double* __restrict__ cg, double* __restrict__ ch, double* __restrict__ lin64,
              double* __restrict__ viol_part, int* flags) {
  __shared__ double red[kBlock / kWave];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double viol = 0.0;
  if (i < n_c) {
    const int4 t = ids[i];
    const d3 X0 = ld3(x, t.x), X1 = ld3(x, t.y), X2 = ld3(x, t.z), X3 = ld3(x, t.w);
    double wv[4];
    d3 diff;
    const bool degenerate = closest_pair(t, i < n_pt, x, diff, wv);
    const double w0 = wv[0], w1 = wv[1], w2 = wv[2], w3 = wv[3];
    const double d = sqrt(dot(diff, diff));
    if (degenerate || !(d > 0.0)) {
      atomicOr(flags, FLAG_DEGENERATE);
      cg[i] = ch[i] = 0.0;
      for (int m = 0; m < 8; ++m) lin64[(long long)m * n_c + i] = 0.0;
    } else {
      const d3 n = mul(diff, 1.0 / d);
      // c_i(x_hat) = d_i(x) + grad d_i(x)^T (x_hat - x) - delta
      const double c = d - delta + w0 * dot(n, sub(ld3(xh, t.x), X0)) + w1 * dot(n, sub(ld3(xh, t.y), X1)) +
                       w2 * dot(n, sub(ld3(xh, t.z), X2)) + w3 * dot(n, sub(ld3(xh, t.w), X3));
      const double l = lam[i], g = gam[i];
      const double s = fmax(0.0, c - l / kappa);                 // slack
      const double gfac = kappa * g * (c - l / kappa - s);       // zero when s > 0
      viol = fmax(0.0, -c);
      cg[i] = gfac;
      ch[i] = kappa * g;
      // the linearization, for the assembly, the energy and the multiplier update: SoA [8][n]
      const double lv[8] = {d, n.x, n.y, n.z, w0, w1, w2, w3};
#pragma unroll
      for (int m = 0; m < 8; ++m) lin64[(long long)m * n_c + i] = lv[m];
    }
  }
  // block max of the violation (FP64)
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) viol = fmax(viol, __shfl_xor(viol, off, kWave));
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = viol;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = red[0];
    for (int w = 1; w < kBlock / kWave; ++w) m = fmax(m, red[w]);
    viol_part[blockIdx.x] = m;
  }
}

__global__ void k_inc_count(const int4* __restrict__ ids, int n_c, int* cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_c) return;
  const int4 t = ids[i];
  atomicAdd(&cnt[t.x], 1); atomicAdd(&cnt[t.y], 1); atomicAdd(&cnt[t.z], 1); atomicAdd(&cnt[t.w], 1);
}

__global__ void k_inc_fill(const int4* __restrict__ ids, int n_c, const int* __restrict__ ptr, int* cursor,
                           int* inc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_c) return;
  const int4 t = ids[i];
  for (int a = 0; a < 4; ++a) {
    const int v = vtx(t, a);
    inc[ptr[v] + atomicAdd(&cursor[v], 1)] = 4 * i + a;
  }
}

// Upper bound on the off-diagonal columns of row r: its elastic columns plus,
// for every incident constraint, its other vertices with a larger id.
__global__ void k_cand_count(const int* __restrict__ erow_ptr, const int* __restrict__ vptr,
                             const int* __restrict__ vinc, const int4* __restrict__ ids, int N, int* ccount) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= N) return;
  int n = erow_ptr[r + 1] - erow_ptr[r] - 1;
  for (int j = vptr[r]; j < vptr[r + 1]; ++j) {
    const int4 t = ids[vinc[j] >> 2];
    n += (t.x > r) + (t.y > r) + (t.z > r) + (t.w > r);
  }
  ccount[r] = n;
}

// One wave per row: gather the row's candidate columns into LDS, sort them by
// rank (stable: rank = #smaller + #equal with a lower index), keep the first
// of each run of equal keys, and write the sorted unique columns back to the
// row's candidate segment.  Rows longer than kCandLds fall back to one lane.
constexpr int kCandLds = 1024;

__device__ inline int wave_excl_scan(int v, int* total) {
  const int lane = threadIdx.x & (kWave - 1);
  int inc = v;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int t = __shfl_up(inc, off, kWave);
    if (lane >= off) inc += t;
  }
  *total = __shfl(inc, kWave - 1, kWave);
  return inc - v;
}

__global__ void __launch_bounds__(kBlock)
k_cand_fill(const int* __restrict__ erow_ptr, const int* __restrict__ ecol, const int* __restrict__ vptr,
            const int* __restrict__ vinc, const int4* __restrict__ ids, int N, const int* __restrict__ cptr,
            int* __restrict__ cand, int* __restrict__ ucount) {
  __shared__ int keys[kBlock / kWave][kCandLds];
  __shared__ int sorted[kBlock / kWave][kCandLds];
  const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const int r = blockIdx.x * (kBlock / kWave) + w;
  if (r >= N) return;   // whole wave leaves together
  const int b = cptr[r], n = cptr[r + 1] - b;
  int* K = keys[w];
  int* S = sorted[w];
  if (n > kCandLds) {
    // rare very long row: one lane, in global memory
    if (lane == 0) {
      int m = 0;
      for (int j = erow_ptr[r] + 1; j < erow_ptr[r + 1]; ++j) cand[b + m++] = ecol[j];
      for (int j = vptr[r]; j < vptr[r + 1]; ++j) {
        const int4 t = ids[vinc[j] >> 2];
        if (t.x > r) cand[b + m++] = t.x;
        if (t.y > r) cand[b + m++] = t.y;
        if (t.z > r) cand[b + m++] = t.z;
        if (t.w > r) cand[b + m++] = t.w;
      }
      for (int j = b + 1; j < b + m; ++j) {
        int key = cand[j];
        int k = j - 1;
        while (k >= b && cand[k] > key) { cand[k + 1] = cand[k]; --k; }
        cand[k + 1] = key;
      }
      int u = 0;
      for (int j = b; j < b + m; ++j)
        if (j == b || cand[j] != cand[j - 1]) cand[b + u++] = cand[j];
      ucount[r] = 1 + u;
    }
    return;
  }
  // gather: elastic columns, then the partners of every incident constraint
  const int e0 = erow_ptr[r] + 1, ne = erow_ptr[r + 1] - e0;
  for (int j = lane; j < ne; j += kWave) K[j] = ecol[e0 + j];
  int m = ne;
  for (int j0 = vptr[r]; j0 < vptr[r + 1]; j0 += kWave) {
    const int j = j0 + lane;
    int4 t = make_int4(-1, -1, -1, -1);
    if (j < vptr[r + 1]) t = ids[vinc[j] >> 2];
    const int cnt = (t.x > r) + (t.y > r) + (t.z > r) + (t.w > r);
    int tot;
    int o = m + wave_excl_scan(cnt, &tot);
    if (t.x > r) K[o++] = t.x;
    if (t.y > r) K[o++] = t.y;
    if (t.z > r) K[o++] = t.z;
    if (t.w > r) K[o++] = t.w;
    m += tot;
  }
  __builtin_amdgcn_wave_barrier();
  // stable rank sort
  for (int i = lane; i < m; i += kWave) {
    const int key = K[i];
    int rank = 0;
    for (int j = 0; j < m; ++j) {
      const int kj = K[j];
      rank += (kj < key) || (kj == key && j < i);
    }
    S[rank] = key;
  }
  __builtin_amdgcn_wave_barrier();
  // unique, in order
  int u = 0;
  for (int i0 = 0; i0 < m; i0 += kWave) {
    const int i = i0 + lane;
    const int keep = (i < m) && (i == 0 || S[i] != S[i - 1]);
    int tot;
    const int o = u + wave_excl_scan(keep, &tot);
    if (keep) cand[b + o] = S[i];
    u += tot;
  }
  if (lane == 0) ucount[r] = 1 + u;
}

// Write the merged row (diagonal first) and, for each slot, the static elastic
// slot with the same (row, col), or -1 for a contact-only block.
__global__ void k_merged_write(const int* __restrict__ cand, const int* __restrict__ cptr,
                               const int* __restrict__ row_ptr, const int* __restrict__ erow_ptr,
                               const int* __restrict__ ecol, int N, int* col, int* eslot) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= N) return;
  const int o = row_ptr[r], n = row_ptr[r + 1] - o;
  col[o] = r;
  eslot[o] = erow_ptr[r];
  int ej = erow_ptr[r] + 1;
  const int ee = erow_ptr[r + 1];
  const int b = cptr[r];
  for (int j = 1; j < n; ++j) {
    const int c = cand[b + j - 1];
    col[o + j] = c;
    while (ej < ee && ecol[ej] < c) ++ej;
    eslot[o + j] = (ej < ee && ecol[ej] == c) ? ej : -1;
  }
}

__device__ inline int find_slot(const int* __restrict__ row_ptr, const int* __restrict__ col, int r, int c) {
  int lo = row_ptr[r], hi = row_ptr[r + 1] - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (col[mid] < c) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__constant__ int c_pa[10] = {0, 0, 0, 0, 1, 1, 1, 2, 2, 3};
__constant__ int c_pb[10] = {0, 1, 2, 3, 1, 2, 3, 2, 3, 3};

__global__ void k_cmap(const int4* __restrict__ ids, int n_c, const int* __restrict__ row_ptr,
                       const int* __restrict__ col, int* cmap) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 10LL * n_c) return;
  const int c = (int)(i / 10), k = (int)(i % 10);
  const int4 t = ids[c];
  const int va = vtx(t, c_pa[k]), vb = vtx(t, c_pb[k]);
  cmap[i] = find_slot(row_ptr, col, min(va, vb), max(va, vb));
}

// Matching the friction contacts to the constraints with the same stencil
// (the capture copies the constraint rows, and the active-set rebuild keeps
// surviving rows as they are): an open-addressing table of the constraint
// rows (capacity a power of two >= 2 n_c, so a probe always meets an empty
// slot), then per friction contact its constraint (cfr[ci] = fi) or a flag
// that it needs stencils of its own.  Repeated rows are matched by index, not
// by the order in which threads arrive: a contact takes the lowest-numbered
// constraint with its stencil (linear probing keeps every key of one home slot
// in the run that starts there, so the whole run is searched), and of several
// contacts with one stencil the lowest-numbered one is matched.  The matching,
// and so the assembly order, is deterministic.
__device__ inline unsigned stencil_hash(const int4 t) {
  unsigned h = (unsigned)t.x * 0x9E3779B1u;
  h = (h ^ (h >> 15)) + (unsigned)t.y * 0x85EBCA77u;
  h = (h ^ (h >> 13)) + (unsigned)t.z * 0xC2B2AE3Du;
  h = (h ^ (h >> 16)) + (unsigned)t.w * 0x27D4EB2Fu;
  return h ^ (h >> 15);
}

__device__ inline bool same4(const int4 a, const int4 b) { return a.x == b.x && a.y == b.y && a.z == b.z && a.w == b.w; }

__global__ void k_stencil_insert(const int4* __restrict__ ids, int n_c, int* tab, unsigned mask) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_c) return;
  unsigned h = stencil_hash(ids[i]) & mask;
  while (atomicCAS(&tab[h], -1, i) != -1) h = (h + 1) & mask;
}

__global__ void k_friction_match(const int4* __restrict__ fids, int n_f, const int4* __restrict__ ids,
                                 const int* __restrict__ tab, unsigned mask, int* cfr, int* __restrict__ extra) {
  const int fi = blockIdx.x * blockDim.x + threadIdx.x;
  if (fi >= n_f) return;
  const int4 t = fids[fi];
  unsigned h = stencil_hash(t) & mask;
  int found = -1;
  for (int s = tab[h]; s != -1; h = (h + 1) & mask, s = tab[h])
    if (same4(ids[s], t) && (found < 0 || s < found)) found = s;
  // cfr starts at -1 (the largest unsigned value): it ends at the lowest contact
  if (found >= 0) atomicMin(reinterpret_cast<unsigned*>(cfr) + found, (unsigned)fi);
  extra[fi] = found;
}

// A contact keeps stencils of its own unless it is the one its constraint took.
__global__ void k_friction_flag(int n_f, const int* __restrict__ cfr, int* __restrict__ extra) {
  const int fi = blockIdx.x * blockDim.x + threadIdx.x;
  if (fi >= n_f) return;
  const int found = extra[fi];
  extra[fi] = (found >= 0 && cfr[found] == fi) ? 0 : 1;
}

// The unmatched friction contacts, in order, after the constraints in the
// pattern's stencil list (pids[n_c + pos]) and their contact ids (fext[pos]).
__global__ void k_friction_extra(const int4* __restrict__ fids, int n_f, const int* __restrict__ extra,
                                 const int* __restrict__ pos, int n_c, int4* __restrict__ pids,
                                 int* __restrict__ fext) {
  const int fi = blockIdx.x * blockDim.x + threadIdx.x;
  if (fi >= n_f || !extra[fi]) return;
  pids[n_c + pos[fi]] = fids[fi];
  fext[pos[fi]] = fi;
}

// Friction capture (Appendix A, semi-implicit): per contact of the previous
// step, at x^t, the closest-point weights w, the normal n and the coefficient
// coef = mu_f max(0, lambda - kappa (d - delta)) = h^2 mu_f F^t.  FP64 SoA
// [8][n_f]: n (3), w (4), coef.  A degenerate pair contributes nothing.
__global__ void __launch_bounds__(kBlock)
k_friction_capture(const int4* __restrict__ ids, int n_pt, int n_f, const double* __restrict__ x,
                   const double* __restrict__ lam, double kappa, double delta, double mu_f,
                   double* __restrict__ f64) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_f) return;
  double w[4];
  d3 diff;
  const bool degenerate = closest_pair(ids[i], i < n_pt, x, diff, w);
  const double d = sqrt(dot(diff, diff));
  double v[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (!degenerate && d > 0.0) {
    const d3 n = mul(diff, 1.0 / d);
    v[0] = n.x; v[1] = n.y; v[2] = n.z;
    v[3] = w[0]; v[4] = w[1]; v[5] = w[2]; v[6] = w[3];
    v[7] = mu_f * fmax(0.0, lam[i] - kappa * (d - delta));
  }
#pragma unroll
  for (int m = 0; m < 8; ++m) f64[(long long)m * n_f + i] = v[m];
}

// Friction terms at x_hat (IPC's smoothed f_0 of the tangential relative
// displacement, e = eps_v h): with v = sum_a w_a (x_hat_a - x^t_a), u = P v
// (P = I - n n^T), y = |u|, t = u / y,
//   gradient in v:  coef f_1(y)/y u
//   Hessian in v:   coef (f_1(y)/y P + (f_1'(y) - f_1(y)/y) t t^T),
// f_1(y)/y = 1/y and f_1' = 0 for y >= e, 2/e - y/e^2 and 2/e - 2y/e^2 below.
// Its eigenvalues coef f_1/y (tangent, across t), coef f_1' (along t) and 0
// (normal) are never negative, so the SPD projection leaves it unchanged.
// FP64 SoA [13][n_f]: gradient (3), Hessian (6: xx xy xz yy yz zz), weights (4).
__global__ void __launch_bounds__(kBlock)
k_friction_terms(const int4* __restrict__ ids, int n_f, const double* __restrict__ xh,
                 const double* __restrict__ x0, const double* __restrict__ f64, double e,
                 double* __restrict__ fgk) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_f) return;
  const int4 t4 = ids[i];
  const int vv[4] = {t4.x, t4.y, t4.z, t4.w};
  double fv[8];
#pragma unroll
  for (int m = 0; m < 8; ++m) fv[m] = f64[(long long)m * n_f + i];
  d3 v = {0.0, 0.0, 0.0};
#pragma unroll
  for (int a = 0; a < 4; ++a) v = add(v, mul(sub(ld3(xh, vv[a]), ld3(x0, vv[a])), fv[3 + a]));
  const d3 n = {fv[0], fv[1], fv[2]};
  const d3 u = sub(v, mul(n, dot(n, v)));
  const double y = sqrt(dot(u, u));
  const double coef = fv[7];
  const double f1y = y >= e ? 1.0 / y : 2.0 / e - y / (e * e);
  const double f1p = y >= e ? 0.0 : 2.0 / e - 2.0 * y / (e * e);
  const d3 tt = y > 0.0 ? mul(u, 1.0 / y) : d3{0.0, 0.0, 0.0};
  const double g[3] = {coef * f1y * u.x, coef * f1y * u.y, coef * f1y * u.z};
  const double nn[3] = {n.x, n.y, n.z}, tv[3] = {tt.x, tt.y, tt.z};
  const int ri[6] = {0, 0, 0, 1, 1, 2}, ci[6] = {0, 1, 2, 1, 2, 2};
  double out[13];
#pragma unroll
  for (int k = 0; k < 3; ++k) out[k] = g[k];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const int r = ri[k], c = ci[k];
    const double P = (r == c ? 1.0 : 0.0) - nn[r] * nn[c];
    out[3 + k] = coef * (f1y * P + (f1p - f1y) * tv[r] * tv[c]);
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) out[9 + a] = fv[3 + a];
#pragma unroll
  for (int m = 0; m < 13; ++m) fgk[(long long)m * n_f + i] = out[m];
}

}  // namespace

void launch_check_constraints(const int4* ids, int n_c, int N, const double* lam, const double* gam, int* flags,
                              hipStream_t s) {
  if (n_c > 0)
    hipLaunchKernelGGL(k_check_constraints, dim3(div_up(n_c, kBlock)), dim3(kBlock), 0, s, ids, n_c, N, lam, gam,
                       flags);
}

void launch_contact_lin(const int4* ids, int n_pt, int n_c, const double* x, const double* xh, const double* lam,
                        const double* gam, double kappa, double delta, double* cg, double* ch, double* lin64,
                        double* viol_part, int* flags, hipStream_t s) {
  if (n_c > 0)
    hipLaunchKernelGGL(k_contact_lin, dim3(div_up(n_c, kBlock)), dim3(kBlock), 0, s, ids, n_pt, n_c, x, xh, lam,
                       gam, kappa, delta, cg, ch, lin64, viol_part, flags);
}

void launch_vertex_incidence_count(const int4* ids, int n_c, int* cnt, hipStream_t s) {
  if (n_c > 0) hipLaunchKernelGGL(k_inc_count, dim3(div_up(n_c, kBlock)), dim3(kBlock), 0, s, ids, n_c, cnt);
}

void launch_vertex_incidence_fill(const int4* ids, int n_c, const int* ptr, int* cursor, int* inc, hipStream_t s) {
  if (n_c > 0)
    hipLaunchKernelGGL(k_inc_fill, dim3(div_up(n_c, kBlock)), dim3(kBlock), 0, s, ids, n_c, ptr, cursor, inc);
}

void launch_candidate_count(const int* erow_ptr, const int* vptr, const int* vinc, const int4* ids, int N,
                            int* ccount, hipStream_t s) {
  hipLaunchKernelGGL(k_cand_count, dim3(div_up(N, kBlock)), dim3(kBlock), 0, s, erow_ptr, vptr, vinc, ids, N,
                     ccount);
}

void launch_candidate_fill(const int* erow_ptr, const int* ecol, const int* vptr, const int* vinc, const int4* ids,
                           int N, const int* cptr, int* cand, int* ucount, hipStream_t s) {
  hipLaunchKernelGGL(k_cand_fill, dim3(div_up(N, kBlock / kWave)), dim3(kBlock), 0, s, erow_ptr, ecol, vptr, vinc, ids,
                     N, cptr, cand, ucount);
}

void launch_merged_write(const int* cand, const int* cptr, const int* row_ptr, const int* erow_ptr, const int* ecol,
                         int N, int* col, int* eslot, hipStream_t s) {
  hipLaunchKernelGGL(k_merged_write, dim3(div_up(N, kBlock)), dim3(kBlock), 0, s, cand, cptr, row_ptr, erow_ptr,
                     ecol, N, col, eslot);
}

void launch_cmap(const int4* ids, int n_c, const int* row_ptr, const int* col, int* cmap, hipStream_t s) {
  if (n_c > 0)
    hipLaunchKernelGGL(k_cmap, dim3(div_up(10LL * n_c, kBlock)), dim3(kBlock), 0, s, ids, n_c, row_ptr, col, cmap);
}

void launch_friction_capture(const int4* ids, int n_pt, int n_f, const double* x, const double* lam, double kappa,
                             double delta, double mu_f, double* f64, hipStream_t s) {
  if (n_f > 0)
    hipLaunchKernelGGL(k_friction_capture, dim3(div_up(n_f, kBlock)), dim3(kBlock), 0, s, ids, n_pt, n_f, x, lam,
                       kappa, delta, mu_f, f64);
}

void launch_stencil_insert(const int4* ids, int n_c, int* tab, unsigned mask, hipStream_t s) {
  if (n_c > 0)
    hipLaunchKernelGGL(k_stencil_insert, dim3(div_up(n_c, kBlock)), dim3(kBlock), 0, s, ids, n_c, tab, mask);
}

void launch_friction_match(const int4* fids, int n_f, const int4* ids, const int* tab, unsigned mask, int* cfr,
                           int* extra, hipStream_t s) {
  if (n_f > 0) {
    hipLaunchKernelGGL(k_friction_match, dim3(div_up(n_f, kBlock)), dim3(kBlock), 0, s, fids, n_f, ids, tab, mask,
                       cfr, extra);
    hipLaunchKernelGGL(k_friction_flag, dim3(div_up(n_f, kBlock)), dim3(kBlock), 0, s, n_f, (const int*)cfr, extra);
  }
}

void launch_friction_extra(const int4* fids, int n_f, const int* extra, const int* pos, int n_c, int4* pids,
                           int* fext, hipStream_t s) {
  if (n_f > 0)
    hipLaunchKernelGGL(k_friction_extra, dim3(div_up(n_f, kBlock)), dim3(kBlock), 0, s, fids, n_f, extra, pos, n_c,
                       pids, fext);
}

void launch_friction_terms(const int4* ids, int n_f, const double* xh, const double* x0, const double* f64, double e,
                           double* fgk, hipStream_t s) {
  if (n_f > 0)
    hipLaunchKernelGGL(k_friction_terms, dim3(div_up(n_f, kBlock)), dim3(kBlock), 0, s, ids, n_f, xh, x0, f64, e,
                       fgk);
}

}  // namespace bfal
