// Block-Jacobi preconditioned CG (the paper's linear solver: CG with a 3x3
// block-Jacobi preconditioner on the symmetric BSR matrix), run on the
// symmetrically scaled system H_hat = L^{-1} H L^{-T} (D_v = L_v L_v^T), whose
// diagonal blocks are identities.  In exact arithmetic its iterates are those
// of PCG with z = D^{-1} r on H: p = L^{-T} p_hat, r = L r_hat.
//
// Only the upper off-diagonal blocks of H_hat are stored and each is read once
// per iteration.  The symmetric product q = H_hat p runs in two phases with no
// atomics: the SpMV kernel forms, per row r, q_row = p_r + sum_{c>r} B_rc p_c
// and writes every block's transposed product t_j = B_rc^T p_r to its own slot
// of tbuf; the update kernel completes q_c = q_row_c + sum of t_j over the
// blocks j in column c (the transpose index, in increasing source row).
// p^T H_hat p = sum_r p_r.(p_r + 2 sum_{c>r} B_rc p_c) is formed in the first
// phase.  One iteration is three kernels on one stream, with no host round trip:
//   spmv      q_row, tbuf, p^T q (FP64)
//   update    q = q_row + transposed sums; alpha = rho / p^T q; x += alpha p,
//             r -= alpha q; rho' = r^T r (FP64); every check_every iterations
//             also |L r|^2, the unscaled residual norm squared.
//   direction beta = rho' / rho, convergence test, p = r + beta p.
// Grid-wide sums: every workgroup writes one FP64 partial per quantity, and
// every workgroup of the *next* kernel re-sums all partials in the same fixed
// order, so every workgroup derives bit-identical scalars without any device
// fence or atomic (kernel boundaries make the partials visible).  Scalars the
// host polls (iteration count, convergence flag, residual) are written by
// workgroup 0 only, into fields no other workgroup of that kernel reads.
// After the flag is set every kernel returns at entry, so the host enqueues
// iterations in batches and polls between batches.
#include "common.h"

namespace bfal {

namespace {

constexpr int kVecBlock = 1024;                    // threads per workgroup of the vector kernels
constexpr int kGridVec = 256;                      // workgroups of the vector kernels (partials per sum)
constexpr int kSpmvBlock = 512;                    // threads per workgroup of the SpMV
constexpr int kGridSpmv = 1024;                    // workgroups of the SpMV (multiple of 8 XCDs)
constexpr int kGroup = 8;                          // lanes per BSR row in the SpMV
constexpr int kRowsPerPass = kSpmvBlock / kGroup;  // rows per workgroup pass in the SpMV

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

// Fixed-order sum of part[0..n) by the whole workgroup (same value in every workgroup).
template <int NT>
__device__ inline double sum_parts(const double* __restrict__ part, int n) {
  double s = 0.0;
  for (int k = threadIdx.x; k < n; k += NT) s += part[k];
  return block_sum_all<NT>(s);
}

// Write this workgroup's partial (thread 0).
__device__ inline void put_part(double* part, double v) {
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}

// XCD-aware workgroup index: dispatch ids round-robin over the 8 XCDs, so give
// each XCD one contiguous range of rows (better L2 reuse of the gathered p).
__device__ inline int xcd_block() {
  const int nb = gridDim.x;
  const int b = blockIdx.x;
  return (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
}

// Smallest row r with frow_ptr[r] >= target (N when none); the last range ends at N.
__device__ inline int first_row_at(const int* __restrict__ frow_ptr, int N, long long target) {
  int lo = 0, hi = N;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (frow_ptr[mid] < target) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__global__ void __launch_bounds__(kSpmvBlock)
k_spmv(int N, const int* __restrict__ urow_ptr, const int* __restrict__ ucol, const float* __restrict__ uv,
       long long st, const float* __restrict__ p, float* __restrict__ qrow, float* __restrict__ tbuf,
       double* __restrict__ part_pq, const PcgScalars* __restrict__ sc) {
  if (sc->done) return;
  // rows [r0, r1) hold about 1/gridDim.x of the stored blocks (rows with
  // contact blocks are longer, and they cluster at the interfaces)
  const int lb = xcd_block();
  const long long nnz = urow_ptr[N];
  const int r0 = first_row_at(urow_ptr, N, (nnz * lb) / gridDim.x);
  const int r1 = (lb == (int)gridDim.x - 1) ? N : first_row_at(urow_ptr, N, (nnz * (lb + 1)) / gridDim.x);
  const int g = threadIdx.x / kGroup, k = threadIdx.x % kGroup;
  double dot = 0.0;
  for (int rb = r0; rb < r1; rb += kRowsPerPass) {
    const int r = rb + g;
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, pr0 = 0.f, pr1 = 0.f, pr2 = 0.f;
    if (r < r1) {
      pr0 = p[3LL * r]; pr1 = p[3LL * r + 1]; pr2 = p[3LL * r + 2];
      const int je = urow_ptr[r + 1];
      for (int j = urow_ptr[r] + k; j < je; j += kGroup) {
        const int c = ucol[j];
        float b[9];
#pragma unroll
        for (int m = 0; m < 9; ++m) b[m] = uv[m * st + j];
        const float pc0 = p[3LL * c], pc1 = p[3LL * c + 1], pc2 = p[3LL * c + 2];
        a0 += b[0] * pc0 + b[1] * pc1 + b[2] * pc2;
        a1 += b[3] * pc0 + b[4] * pc1 + b[5] * pc2;
        a2 += b[6] * pc0 + b[7] * pc1 + b[8] * pc2;
        float* t = tbuf + 3LL * j;
        t[0] = b[0] * pr0 + b[3] * pr1 + b[6] * pr2;
        t[1] = b[1] * pr0 + b[4] * pr1 + b[7] * pr2;
        t[2] = b[2] * pr0 + b[5] * pr1 + b[8] * pr2;
      }
    }
#pragma unroll
    for (int off = kGroup / 2; off > 0; off >>= 1) {
      a0 += __shfl_xor(a0, off, kGroup);
      a1 += __shfl_xor(a1, off, kGroup);
      a2 += __shfl_xor(a2, off, kGroup);
    }
    if (r < r1 && k == 0) {
      qrow[3LL * r] = pr0 + a0;   // identity diagonal block + upper part
      qrow[3LL * r + 1] = pr1 + a1;
      qrow[3LL * r + 2] = pr2 + a2;
      dot += (double)pr0 * pr0 + (double)pr1 * pr1 + (double)pr2 * pr2 +
             2.0 * ((double)pr0 * a0 + (double)pr1 * a1 + (double)pr2 * a2);
    }
  }
  put_part(part_pq, block_sum_all<kSpmvBlock>(dot));
}

__global__ void __launch_bounds__(kVecBlock)
k_update(int N, const float* __restrict__ Lf, float* __restrict__ x, float* __restrict__ r,
         const float* __restrict__ p, const float* __restrict__ qrow, const float* __restrict__ tbuf,
         const int* __restrict__ tptr, const int* __restrict__ tidx, const double* __restrict__ part_pq, int n_pq,
         double* __restrict__ part_rr, double* __restrict__ part_rt, PcgScalars* __restrict__ sc) {
  if (sc->done) return;
  const int k = sc->iter3;
  const double rho = sum_parts<kVecBlock>(part_rr + (k & 1) * kGridVec, gridDim.x);
  const double pq = sum_parts<kVecBlock>(part_pq, n_pq);
  if (blockIdx.x == 0 && threadIdx.x == 0) sc->iter2 = k;
  if (!(pq > 0.0)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      sc->flags |= FLAG_BREAKDOWN;
      sc->done = 3;
    }
    return;
  }
  const float alpha = (float)(rho / pq);
  const bool check = ((k + 1) % sc->check_every) == 0;
  double rr = 0.0, rt = 0.0;
  for (int v = blockIdx.x * kVecBlock + threadIdx.x; v < N; v += gridDim.x * kVecBlock) {
    const long long o = 3LL * v;
    float q0 = qrow[o], q1 = qrow[o + 1], q2 = qrow[o + 2];
    for (int i = tptr[v]; i < tptr[v + 1]; ++i) {
      const float* t = tbuf + 3LL * tidx[i];
      q0 += t[0];
      q1 += t[1];
      q2 += t[2];
    }
    const float r0 = r[o] - alpha * q0, r1 = r[o + 1] - alpha * q1, r2 = r[o + 2] - alpha * q2;
    x[o] += alpha * p[o];
    x[o + 1] += alpha * p[o + 1];
    x[o + 2] += alpha * p[o + 2];
    r[o] = r0;
    r[o + 1] = r1;
    r[o + 2] = r2;
    rr += (double)r0 * r0 + (double)r1 * r1 + (double)r2 * r2;
    if (check) {
      const float* l = Lf + 6LL * v;
      const double t0 = (double)l[0] * r0;
      const double t1 = (double)l[1] * r0 + (double)l[2] * r1;
      const double t2 = (double)l[3] * r0 + (double)l[4] * r1 + (double)l[5] * r2;
      rt += t0 * t0 + t1 * t1 + t2 * t2;
    }
  }
  put_part(part_rr + ((k + 1) & 1) * kGridVec, block_sum_all<kVecBlock>(rr));
  put_part(part_rt, block_sum_all<kVecBlock>(rt));
}

__global__ void __launch_bounds__(kVecBlock)
k_direction(int N4, const float* __restrict__ r, float* __restrict__ p, const double* __restrict__ part_rr,
            const double* __restrict__ part_rt, PcgScalars* __restrict__ sc) {
  if (sc->done) return;
  const int k = sc->iter2;
  const double rho_old = sum_parts<kVecBlock>(part_rr + (k & 1) * kGridVec, gridDim.x);
  const double rho_new = sum_parts<kVecBlock>(part_rr + ((k + 1) & 1) * kGridVec, gridDim.x);
  const bool check = ((k + 1) % sc->check_every) == 0;
  const double rt = check ? sum_parts<kVecBlock>(part_rt, gridDim.x) : 0.0;
  const bool converged = (check && rt <= sc->tol2 * sc->bb) || rho_new == 0.0;
  const bool capped = (k + 1) >= sc->max_iter;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc->iter3 = k + 1;
    sc->rho = rho_new;
    if (check) sc->rr_true = rt;
    if (converged) sc->done = 1;
    else if (capped) sc->done = 2;
  }
  if (converged || capped) return;
  const float beta = (float)(rho_new / rho_old);
  const int nf4 = 3 * (N4 / 4);
  const float4* r4 = reinterpret_cast<const float4*>(r);
  float4* p4 = reinterpret_cast<float4*>(p);
  for (int i = blockIdx.x * kVecBlock + threadIdx.x; i < nf4; i += gridDim.x * kVecBlock) {
    const float4 rv = r4[i];
    float4 pv = p4[i];
    pv.x = rv.x + beta * pv.x; pv.y = rv.y + beta * pv.y; pv.z = rv.z + beta * pv.z; pv.w = rv.w + beta * pv.w;
    p4[i] = pv;
  }
}

__global__ void __launch_bounds__(kVecBlock)
k_init(int N4, const float* __restrict__ bhat, float* __restrict__ x, float* __restrict__ r, float* __restrict__ p,
       double* __restrict__ part_rr) {
  double rr = 0.0;
  const long long n3 = 3LL * N4;
  for (long long i = (long long)blockIdx.x * kVecBlock + threadIdx.x; i < n3; i += (long long)gridDim.x * kVecBlock) {
    const float b = bhat[i];
    x[i] = 0.f;
    r[i] = b;
    p[i] = b;
    rr += (double)b * b;
  }
  put_part(part_rr, block_sum_all<kVecBlock>(rr));   // iteration 0 reads slot (0 & 1) = 0
}

__global__ void __launch_bounds__(kBlock)
k_init_scalars(const double* __restrict__ bb_part, int nbb, PcgScalars* sc, double tol, int max_iter,
               int check_every) {
  const double bb = sum_parts<kBlock>(bb_part, nbb);
  if (threadIdx.x == 0) {
    sc->bb = bb;
    sc->rr_true = bb;
    sc->rho = 0.0;
    sc->tol2 = tol * tol;
    sc->iter2 = 0;
    sc->iter3 = 0;
    sc->max_iter = max_iter;
    sc->check_every = check_every > 0 ? check_every : 1;
    sc->flags = 0;
    sc->done = (bb == 0.0) ? 1 : (max_iter <= 0 ? 2 : 0);
  }
}

// p = L^{-T} p_hat in FP64 and the per-workgroup max |p|.
__global__ void __launch_bounds__(kVecBlock)
k_finish(int N, const float* __restrict__ Linv, const float* __restrict__ x, double* __restrict__ pout,
         double* __restrict__ part) {
  double m = 0.0;
  for (int v = blockIdx.x * kVecBlock + threadIdx.x; v < N; v += gridDim.x * kVecBlock) {
    const float* l = Linv + 6LL * v;
    const double x0 = x[3LL * v], x1 = x[3LL * v + 1], x2 = x[3LL * v + 2];
    const double p0 = (double)l[0] * x0 + (double)l[1] * x1 + (double)l[3] * x2;
    const double p1 = (double)l[2] * x1 + (double)l[4] * x2;
    const double p2 = (double)l[5] * x2;
    pout[3LL * v] = p0;
    pout[3LL * v + 1] = p1;
    pout[3LL * v + 2] = p2;
    m = fmax(m, fmax(fabs(p0), fmax(fabs(p1), fabs(p2))));
  }
  const double s = block_max_all<kVecBlock>(m);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
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

inline int pad4(int N) { return (N + 3) & ~3; }

inline int vec_grid(int N) {
  int g = div_up(N, kVecBlock);
  return g < 1 ? 1 : (g > kGridVec ? kGridVec : g);
}

inline int spmv_grid(int N) {
  int g = div_up(N, kRowsPerPass);
  if (g > kGridSpmv) g = kGridSpmv;
  return ((g + 7) / 8) * 8;
}

}  // namespace

// Vectors x, r, p, q, b_hat and the factor L hold pad4(N) nodes; the pad
// entries are zero and stay zero (the SpMV writes q for the N real rows only).
// Partials layout: [0, 2*kGridVec) r^T r of two consecutive iterations,
// [2k, 3k) |L r|^2, [3k, 3k + kGridSpmv) p^T q  (k = kGridVec).
int pcg_partials_needed(int N) {
  (void)N;
  return 3 * kGridVec + kGridSpmv + 64;
}

void launch_pcg_init(int N, const float* bhat, float* x, float* r, float* p, double* part, const double* bb_part,
                     int nbb, PcgScalars* sc, double tol, int max_iter, int check_every, hipStream_t s) {
  hipLaunchKernelGGL(k_init, dim3(vec_grid(N)), dim3(kVecBlock), 0, s, pad4(N), bhat, x, r, p, part);
  hipLaunchKernelGGL(k_init_scalars, dim3(1), dim3(kBlock), 0, s, bb_part, nbb, sc, tol, max_iter, check_every);
}

void launch_pcg_spmv(int N, const int* urow_ptr, const int* ucol, const float* uvals, long long ustride,
                     const float* p, float* qrow, float* tbuf, double* part, PcgScalars* sc, hipStream_t s) {
  hipLaunchKernelGGL(k_spmv, dim3(spmv_grid(N)), dim3(kSpmvBlock), 0, s, N, urow_ptr, ucol, uvals, ustride, p, qrow,
                     tbuf, part + 3 * kGridVec, (const PcgScalars*)sc);
}

void launch_pcg_vector_ops(int N, const float* Lf, float* x, float* r, float* p, const float* qrow,
                           const float* tbuf, const int* tptr, const int* tidx, double* part, PcgScalars* sc,
                           hipStream_t s) {
  const int gv = vec_grid(N);
  hipLaunchKernelGGL(k_update, dim3(gv), dim3(kVecBlock), 0, s, N, Lf, x, r, (const float*)p, qrow, tbuf, tptr, tidx,
                     (const double*)(part + 3 * kGridVec), spmv_grid(N), part, part + 2 * kGridVec, sc);
  hipLaunchKernelGGL(k_direction, dim3(gv), dim3(kVecBlock), 0, s, pad4(N), (const float*)r, p, (const double*)part,
                     (const double*)(part + 2 * kGridVec), sc);
}

void launch_pcg_finish(int N, const float* Linv, const float* x, double* pout, double* part, PcgScalars* sc,
                       const double* viol_part, int nviol, hipStream_t s) {
  const int g = vec_grid(N);
  hipLaunchKernelGGL(k_finish, dim3(g), dim3(kVecBlock), 0, s, N, Linv, x, pout, part);
  hipLaunchKernelGGL(k_finish_scalars, dim3(1), dim3(kBlock), 0, s, (const double*)part, g, viol_part, nviol, sc);
}

}  // namespace bfal
