// Row-owner assembly of G and of the upper 3x3-block matrix H, one thread per
// row, in a fixed order (no atomics on the matrix, bitwise reproducible):
//   - elastic blocks: sum of the per-tet contributions of each static slot, in
//     the slot's precomputed (tet, pair) order;
//   - inertia (Section 3): diagonal += m_v I, G_v += m_v (x_hat_v - x_tilde_v);
//   - AL contact terms of the contact loop of Algorithm 2, for every incident
//     constraint in increasing id: G_a += gfac w_a n and block(a, b) +=
//     hfac w_a w_b n n^T (hfac = kappa gamma, kept also for inactive pairs);
//   - friction terms of the previous step's contacts (Appendix A): G_a +=
//     w_a g and block(a, b) += w_a w_b K with the contact's gradient g and 3x3
//     Hessian K in the relative displacement, at the incidences of the
//     constraint with the same stencil (cfr) or, for a contact without one,
//     at its own stencil listed after the constraints (fext);
//   - moving-boundary elimination (Section 5.3): G_v = 0 and every entry in
//     the rows and columns of a fixed node zeroed except its scalar diagonals.
// Then the block-Jacobi preconditioner (the paper's 3x3 block-Jacobi PCG) is
// applied symmetrically: each diagonal block is factored D_v = L_v L_v^T and
// the off-diagonal blocks are scaled to L_r^{-1} H_rc L_c^{-T}, so the solver
// runs CG on a matrix whose diagonal blocks are identities.  Only the upper
// off-diagonal scaled blocks are stored (in slices of 64 rows, see
// k_slice_widths), plus, per row, references to the upper blocks of its column
// through which the SpMV gathers the lower half.
#include "common.h"

namespace bfal {

namespace {

__device__ inline int vtx(const int4& t, int a) { return a == 0 ? t.x : a == 1 ? t.y : a == 2 ? t.z : t.w; }

__device__ inline int find_slot(const int* __restrict__ col, int lo, int hi, int c) {
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (col[mid] < c) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Slot index of the local vertex pair (i, j), i < j, in a stencil's ten
// pairs (0,0),(0,1),(0,2),(0,3),(1,1),(1,2),(1,3),(2,2),(2,3),(3,3).
__device__ inline int pair_index(int i, int j) { return (i == 0 ? 0 : i == 1 ? 4 : i == 2 ? 7 : 9) + (j - i); }

// Friction contact fi at vertex slot a of its stencil t (whose ten pair
// slots are cs), into row r's diagonal d, gradient g and upper blocks.
__device__ inline void add_friction(int fi, int a, const int4& t, int r, const int* __restrict__ cs, int n_f,
                                    const double* __restrict__ fgk, double* vals, double d[6], double g[3]) {
  double K[6], w[4];
#pragma unroll
  for (int k = 0; k < 6; ++k) K[k] = fgk[(3LL + k) * n_f + fi];
#pragma unroll
  for (int k = 0; k < 4; ++k) w[k] = fgk[(9LL + k) * n_f + fi];
  const double wa = w[a];
#pragma unroll
  for (int k = 0; k < 3; ++k) g[k] += wa * fgk[(long long)k * n_f + fi];
  const double saa = wa * wa;
#pragma unroll
  for (int k = 0; k < 6; ++k) d[k] += saa * K[k];
  for (int b = 0; b < 4; ++b) {
    const int vb = vtx(t, b);
    if (b == a || vb < r) continue;
    const int s = cs[pair_index(min(a, b), max(a, b))];
    const double sab = wa * w[b];
    double* v = vals + 9LL * s;
    v[0] += sab * K[0]; v[1] += sab * K[1]; v[2] += sab * K[2];
    v[3] += sab * K[1]; v[4] += sab * K[3]; v[5] += sab * K[4];
    v[6] += sab * K[2]; v[7] += sab * K[4]; v[8] += sab * K[5];
  }
}

// Elastic sums of the merged pattern's off-diagonal slots, one thread per
// slot: the slot's range of (tet, pair) contributions in FP64, in that order,
// written to vals before the row owners add the contact and friction terms
// (so every block is summed in the same order as by its row owner alone); a
// slot without a static elastic part (contact only) starts at zero.  A static
// slot es is a diagonal one, left to the row owner, when erow_ptr[ecol[es]]
// == es (the static pattern holds each row's diagonal first).  Threads beyond
// the merged pattern's row_ptr[N] slots return.
__global__ void __launch_bounds__(kBlock)
k_offdiag_sums(int N, long long cap, const int* __restrict__ row_ptr, const int* __restrict__ eslot,
               const int* __restrict__ erow_ptr, const int* __restrict__ ecol, const int* __restrict__ ecptr,
               const double* __restrict__ staging, double* __restrict__ vals) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cap || j >= row_ptr[N]) return;
  const int es = eslot[j];
  if (es >= 0 && erow_ptr[ecol[es]] == es) return;
  double b[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (es >= 0) {
    for (int q = ecptr[es]; q < ecptr[es + 1]; ++q) {
      const double* st = staging + 9LL * q;
#pragma unroll
      for (int k = 0; k < 9; ++k) b[k] += st[k];
    }
  }
  double* v = vals + 9 * j;
#pragma unroll
  for (int k = 0; k < 9; ++k) v[k] = b[k];
}

// All sums, the factor L and the right-hand side in FP64; the blocks stay
// FP64 (vals) until the sliced storage rounds the scaled ones once.
__global__ void __launch_bounds__(kBlock)
k_assemble_rows(int N, const int* __restrict__ row_ptr, const int* __restrict__ col, const int* __restrict__ eslot,
                const int* __restrict__ ecptr, const double* __restrict__ staging, const int* __restrict__ vptr,
                const int* __restrict__ vinc, const int4* __restrict__ ids, const int* __restrict__ cslot, int n_c,
                const double* __restrict__ lin64,
                const double* __restrict__ cg, const double* __restrict__ ch, int n_f,
                const double* __restrict__ fgk, const int* __restrict__ cfr, const int* __restrict__ fext,
                const double* __restrict__ mass, const double* __restrict__ xh, const double* __restrict__ xt,
                const uint8_t* __restrict__ fixed, double* __restrict__ vals, float* __restrict__ grad,
                float* __restrict__ Lf, double* __restrict__ Linv, float* __restrict__ bhat,
                double* __restrict__ bb_part, int* flags) {
  __shared__ double red[kBlock / kWave];
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  double bb = 0.0;
  if (r < N) {
    const int o = row_ptr[r], n = row_ptr[r + 1] - o;
    // diagonal: elastic sum (symmetric 6 + gradient 3 per contribution)
    double d[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, g[3] = {0.0, 0.0, 0.0};
    {
      const int es = eslot[o];
      for (int j = ecptr[es]; j < ecptr[es + 1]; ++j) {
        const double* s = staging + 9LL * j;
#pragma unroll
        for (int k = 0; k < 6; ++k) d[k] += s[k];
#pragma unroll
        for (int k = 0; k < 3; ++k) g[k] += s[6 + k];
      }
    }
    // (the off-diagonal elastic sums are in vals already: k_offdiag_sums)
    // inertia
    const double m = mass[r];
    d[0] += m; d[3] += m; d[5] += m;
#pragma unroll
    for (int k = 0; k < 3; ++k) g[k] += m * (xh[3LL * r + k] - xt[3LL * r + k]);
    // AL contact terms of the incident constraints, then friction terms
    for (int j = vptr[r]; j < vptr[r + 1]; ++j) {
      const int ci = vinc[j] >> 2, a = vinc[j] & 3;
      const int4 t = ids[ci];
      const int* cs = cslot + 10LL * ci;
      if (ci >= n_c) {
        add_friction(fext[ci - n_c], a, t, r, cs, n_f, fgk, vals, d, g);
        continue;
      }
      if (n_f > 0) {
        const int fi = cfr[ci];
        if (fi >= 0) add_friction(fi, a, t, r, cs, n_f, fgk, vals, d, g);
      }
      // normal n and weights w from the linearization (SoA rows 1-3 and 4-7)
      const double n0 = lin64[1LL * n_c + ci], n1 = lin64[2LL * n_c + ci], n2 = lin64[3LL * n_c + ci];
      const double w[4] = {lin64[4LL * n_c + ci], lin64[5LL * n_c + ci], lin64[6LL * n_c + ci],
                           lin64[7LL * n_c + ci]};
      const double gf = cg[ci], hf = ch[ci];
      const double wa = w[a];
      g[0] += gf * wa * n0; g[1] += gf * wa * n1; g[2] += gf * wa * n2;
      const double saa = hf * wa * wa;
      d[0] += saa * n0 * n0; d[1] += saa * n0 * n1; d[2] += saa * n0 * n2;
      d[3] += saa * n1 * n1; d[4] += saa * n1 * n2; d[5] += saa * n2 * n2;
      for (int b = 0; b < 4; ++b) {
        const int vb = vtx(t, b);
        if (b == a || vb < r) continue;
        const int s = cs[pair_index(min(a, b), max(a, b))];
        const double sab = hf * wa * w[b];
        double* v = vals + 9LL * s;
        v[0] += sab * n0 * n0; v[1] += sab * n0 * n1; v[2] += sab * n0 * n2;
        v[3] += sab * n1 * n0; v[4] += sab * n1 * n1; v[5] += sab * n1 * n2;
        v[6] += sab * n2 * n0; v[7] += sab * n2 * n1; v[8] += sab * n2 * n2;
      }
    }
    // moving-boundary elimination
    const bool fr = fixed[r] != 0;
    if (fr) {
      g[0] = g[1] = g[2] = 0.0;
      d[1] = d[2] = d[4] = 0.0;
    }
    for (int j = 1; j < n; ++j) {
      if (fr || fixed[col[o + j]]) {
        double* v = vals + 9LL * (o + j);
#pragma unroll
        for (int k = 0; k < 9; ++k) v[k] = 0.0;
      }
    }
    double* v = vals + 9LL * o;
    v[0] = d[0]; v[1] = d[1]; v[2] = d[2];
    v[3] = d[1]; v[4] = d[3]; v[5] = d[4];
    v[6] = d[2]; v[7] = d[4]; v[8] = d[5];
    grad[3LL * r] = (float)g[0]; grad[3LL * r + 1] = (float)g[1]; grad[3LL * r + 2] = (float)g[2];
    bb = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
    // Cholesky D = L L^T and M = L^{-1} (both lower triangular, 6 entries)
    const double q00 = d[0];
    bool ok = q00 > 0.0;
    const double L00 = ok ? sqrt(q00) : 1.0;
    const double L10 = d[1] / L00, L20 = d[2] / L00;
    const double q11 = d[3] - L10 * L10;
    ok = ok && q11 > 0.0;
    const double L11 = q11 > 0.0 ? sqrt(q11) : 1.0;
    const double L21 = (d[4] - L20 * L10) / L11;
    const double q22 = d[5] - L20 * L20 - L21 * L21;
    ok = ok && q22 > 0.0;
    const double L22 = q22 > 0.0 ? sqrt(q22) : 1.0;
    if (!ok) atomicOr(flags, FLAG_NOT_SPD);
    const double M00 = 1.0 / L00, M11 = 1.0 / L11, M22 = 1.0 / L22;
    const double M10 = -L10 * M00 * M11;
    const double M21 = -L21 * M11 * M22;
    const double M20 = -(L20 * M00 + L21 * M10) * M22;
    // L as FP32 SoA [6][N4] for the solver's residual norm
    const long long N4 = (N + 3) & ~3;
    Lf[r] = (float)L00; Lf[N4 + r] = (float)L10; Lf[2 * N4 + r] = (float)L11; Lf[3 * N4 + r] = (float)L20;
    Lf[4 * N4 + r] = (float)L21; Lf[5 * N4 + r] = (float)L22;
    double* li = Linv + 6LL * r;
    li[0] = M00; li[1] = M10; li[2] = M11; li[3] = M20; li[4] = M21; li[5] = M22;
    // b_hat = L^{-1} b with b = -G, rounded once to FP32
    bhat[3LL * r] = (float)(-(M00 * g[0]));
    bhat[3LL * r + 1] = (float)(-(M10 * g[0] + M11 * g[1]));
    bhat[3LL * r + 2] = (float)(-(M20 * g[0] + M21 * g[1] + M22 * g[2]));
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) bb += __shfl_xor(bb, off, kWave);
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = bb;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kBlock / kWave; ++w) s += red[w];
    bb_part[blockIdx.x] = s;
  }
}

// Transpose index of the upper off-diagonal pattern: for every column c the
// rows r < c holding a block (r, c), sorted (after sort_segments) by r.
__global__ void k_lower_count(int N, const int* __restrict__ row_ptr, const int* __restrict__ col, int* lcnt) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= N) return;
  for (int s = row_ptr[r] + 1; s < row_ptr[r + 1]; ++s) atomicAdd(&lcnt[col[s]], 1);
}

__global__ void k_lower_fill(int N, const int* __restrict__ row_ptr, const int* __restrict__ col,
                             const int* __restrict__ lptr, int* lcur, int* lsrc) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= N) return;
  for (int s = row_ptr[r] + 1; s < row_ptr[r + 1]; ++s) {
    const int c = col[s];
    lsrc[lptr[c] + atomicAdd(&lcur[c], 1)] = r;
  }
}

__device__ inline void scaled_block(const double* __restrict__ mr, const double* __restrict__ b,
                                    const double* __restrict__ mc, double out[3][3]) {
  const double R[3][3] = {{mr[0], 0.0, 0.0}, {mr[1], mr[2], 0.0}, {mr[3], mr[4], mr[5]}};
  const double Cm[3][3] = {{mc[0], 0.0, 0.0}, {mc[1], mc[2], 0.0}, {mc[3], mc[4], mc[5]}};
  double T1[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) T1[i][k] = R[i][0] * b[k] + R[i][1] * b[3 + k] + R[i][2] * b[6 + k];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) out[i][k] = T1[i][0] * Cm[k][0] + T1[i][1] * Cm[k][1] + T1[i][2] * Cm[k][2];
}

// FP32 -> BF16, round to nearest even (NaN kept quiet).
__device__ inline uint32_t bf16_rne(float f) {
  const uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0u;
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

// Sliced storage of the scaled matrix (slices of kSlice consecutive rows, one
// lane per row).  Slice s stores wu(s) = max upper off-diagonal count of its
// rows upper slots and wl(s) = max lower count lower slots, slot k of the row
// in lane l at base + k * kSlice + l (so a wavefront reads slot k of its 64 rows
// contiguously).  Upper slots hold a row's blocks by decreasing column, lower
// slots its column's blocks by increasing source row: on a regular stencil the
// k-th upper slot of row r and the k-th lower slot of row r + d then hold the
// same block, so the SpMV, which visits upper and lower slot k together, reads
// each block twice at nearly the same time.  Shorter rows are padded: an
// upper pad has a zero block and its own row as column; a lower pad points at
// the zero block stored after the last upper slot.
__global__ void k_slice_widths(int N, int nslices, const int* __restrict__ row_ptr, const int* __restrict__ lptr,
                               int* __restrict__ cu, int* __restrict__ cl, int* __restrict__ wmax) {
  const int sl = blockIdx.x * blockDim.x + threadIdx.x;
  if (sl >= nslices) return;
  int wu = 0, wl = 0;
  const int r1 = min(N, (sl + 1) * kSlice);
  for (int r = sl * kSlice; r < r1; ++r) {
    wu = max(wu, row_ptr[r + 1] - row_ptr[r] - 1);
    wl = max(wl, lptr[r + 1] - lptr[r]);
  }
  cu[sl] = wu * kSlice;
  cl[sl] = wl * kSlice;
  atomicMax(&wmax[0], wu);
  atomicMax(&wmax[1], wl);
}

// Upper slots: H_hat_rc = M_r H_rc M_c^T (M = L^{-1}) for every upper
// off-diagonal block, FP32 row-major 9 floats per slot, and when blk16 is set a
// BF16 copy (10 half-words packed two per word, the last one zero).
__global__ void k_sell_upper(int N, int nslices, const int* __restrict__ row_ptr, const int* __restrict__ col,
                             const double* __restrict__ vals, const double* __restrict__ Linv,
                             const int* __restrict__ sbu, float* __restrict__ blk, uint32_t* __restrict__ blk16,
                             int* __restrict__ scol) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nslices * kSlice) return;
  const int sl = r / kSlice, lane = r % kSlice;
  const int base = sbu[sl], wu = (sbu[sl + 1] - base) / kSlice;
  const int o = r < N ? row_ptr[r] : 0;
  const int nu = r < N ? row_ptr[r + 1] - o - 1 : 0;
  const double* mr = Linv + 6LL * (r < N ? r : 0);
  for (int k = 0; k < wu; ++k) {
    const long long e = base + (long long)k * kSlice + lane;
    double hd[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
    int c = r < N ? r : N - 1;
    if (k < nu) {   // decreasing column order
      const int sk = o + nu - k;
      c = col[sk];
      scaled_block(mr, vals + 9LL * sk, Linv + 6LL * c, hd);
    }
    // the scaled block rounded once to FP32 (and from there to BF16)
    float h[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int m = 0; m < 3; ++m) h[i][m] = (float)hd[i][m];
    float* d = blk + 9 * e;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int m = 0; m < 3; ++m) d[3 * i + m] = h[i][m];
    if (blk16) {
      uint32_t* w = blk16 + 5 * e;
      w[0] = bf16_rne(h[0][0]) | (bf16_rne(h[0][1]) << 16);
      w[1] = bf16_rne(h[0][2]) | (bf16_rne(h[1][0]) << 16);
      w[2] = bf16_rne(h[1][1]) | (bf16_rne(h[1][2]) << 16);
      w[3] = bf16_rne(h[2][0]) | (bf16_rne(h[2][1]) << 16);
      w[4] = bf16_rne(h[2][2]);
    }
    scol[e] = c;
  }
  if (r == 0) {   // the zero block the lower pads point at
    const long long z = sbu[nslices];
    for (int m = 0; m < 9; ++m) blk[9 * z + m] = 0.f;
    if (blk16)
      for (int m = 0; m < 5; ++m) blk16[5 * z + m] = 0u;
  }
}

// Lower slots of row c: for every upper block (src, c), src < c, in increasing
// src, the pair (upper slot of the block, src).
__global__ void k_sell_lower(int N, int nslices, const int* __restrict__ row_ptr, const int* __restrict__ col,
                             const int* __restrict__ lptr, const int* __restrict__ lsrc, const int* __restrict__ sbu,
                             const int* __restrict__ sbl, int2* __restrict__ sent) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nslices * kSlice) return;
  const int sl = c / kSlice, lane = c % kSlice;
  const int base = sbl[sl], wl = (sbl[sl + 1] - base) / kSlice;
  const int o = c < N ? lptr[c] : 0;
  const int nl = c < N ? lptr[c + 1] - o : 0;
  const int zero = sbu[nslices];
  for (int k = 0; k < wl; ++k) {
    int2 t = make_int2(zero, c < N ? c : N - 1);
    if (k < nl) {
      const int src = lsrc[o + k];
      const int s = find_slot(col, row_ptr[src] + 1, row_ptr[src + 1] - 1, c);
      const int ks = row_ptr[src + 1] - 1 - s;   // position in src's decreasing upper list
      t = make_int2(sbu[src / kSlice] + ks * kSlice + src % kSlice, src);
    }
    sent[base + (long long)k * kSlice + lane] = t;
  }
}

__global__ void k_row_diag_slots(int N, const int* __restrict__ row_ptr, int* diag) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < N) diag[r] = row_ptr[r];
}

}  // namespace

void launch_assemble_rows(int N, long long cap, const int* row_ptr, const int* col, const int* eslot,
                          const int* erow_ptr, const int* ecol, const int* ecptr, const double* staging,
                          const int* vptr, const int* vinc, const int4* ids, const int* cslot, int n_c,
                          const double* lin64,
                          const double* cg, const double* ch, int n_f, const double* fgk, const int* cfr,
                          const int* fext, const double* mass, const double* xh, const double* xt,
                          const uint8_t* fixed, double* vals, float* grad, float* Lf, double* Linv, float* bhat,
                          double* bb_part, int* flags, hipStream_t s) {
  hipLaunchKernelGGL(k_offdiag_sums, dim3(div_up(cap, kBlock)), dim3(kBlock), 0, s, N, cap, row_ptr, eslot, erow_ptr,
                     ecol, ecptr, staging, vals);
  hipLaunchKernelGGL(k_assemble_rows, dim3(div_up(N, kBlock)), dim3(kBlock), 0, s, N, row_ptr, col, eslot, ecptr,
                     staging, vptr, vinc, ids, cslot, n_c, lin64, cg, ch, n_f, fgk, cfr, fext, mass, xh, xt, fixed, vals,
                     grad, Lf, Linv, bhat, bb_part, flags);
}

void launch_lower_count(int N, const int* row_ptr, const int* col, int* lcnt, hipStream_t s) {
  hipLaunchKernelGGL(k_lower_count, dim3(div_up(N, kBlock)), dim3(kBlock), 0, s, N, row_ptr, col, lcnt);
}

void launch_lower_fill(int N, const int* row_ptr, const int* col, const int* lptr, int* lcur, int* lsrc,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_lower_fill, dim3(div_up(N, kBlock)), dim3(kBlock), 0, s, N, row_ptr, col, lptr, lcur, lsrc);
}

void launch_slice_widths(int N, int nslices, const int* row_ptr, const int* lptr, int* cu, int* cl, int* wmax,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_slice_widths, dim3(div_up(nslices, kBlock)), dim3(kBlock), 0, s, N, nslices, row_ptr, lptr, cu,
                     cl, wmax);
}

void launch_sell_fill(int N, int nslices, const int* row_ptr, const int* col, const double* vals, const double* Linv,
                      const int* lptr, const int* lsrc, const int* sbu, const int* sbl, float* blk, uint32_t* blk16,
                      int* scol, int2* sent, hipStream_t s) {
  const int g = div_up((long long)nslices * kSlice, kBlock);
  hipLaunchKernelGGL(k_sell_upper, dim3(g), dim3(kBlock), 0, s, N, nslices, row_ptr, col, vals, Linv, sbu, blk, blk16,
                     scol);
  hipLaunchKernelGGL(k_sell_lower, dim3(g), dim3(kBlock), 0, s, N, nslices, row_ptr, col, lptr, lsrc, sbu, sbl, sent);
}

void launch_row_diag_slots(int N, const int* row_ptr, int* diag, hipStream_t s) {
  hipLaunchKernelGGL(k_row_diag_slots, dim3(div_up(N, kBlock)), dim3(kBlock), 0, s, N, row_ptr, diag);
}

}  // namespace bfal
