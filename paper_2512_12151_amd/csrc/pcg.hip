// Block-Jacobi preconditioned CG (the paper's linear solver: CG with a 3x3
// block-Jacobi preconditioner on the symmetric BSR matrix), run on the
// symmetrically scaled system H_hat = L^{-1} H L^{-T} (D_v = L_v L_v^T), whose
// diagonal blocks are identities.  In exact arithmetic its iterates are those
// of PCG with z = D^{-1} r on H: p = L^{-T} p_hat, r = L r_hat.
//
// One iteration is three kernels on one stream, with no host round trip:
//   spmv      q = H_hat p = p + sum_c B_rc p_c over the stored off-diagonal
//             blocks of each row (both triangles: a pure gather, no atomics),
//             and p^T q (FP64).
//   update    alpha = rho / p^T q; x += alpha p, r -= alpha q; rho' = r^T r
//             (FP64); every check_every iterations also |L r|^2, the
//             unscaled residual norm squared.
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

constexpr int kGridVec = 1024;                     // workgroups of the vector kernels (partials per sum)
constexpr int kGridSpmv = 1024;                    // workgroups of the SpMV (multiple of 8 XCDs)
constexpr int kGroup = 16;                         // lanes per BSR row in the SpMV
constexpr int kRowsPerPass = kBlock / kGroup;      // rows per workgroup pass in the SpMV

// Sum of v over the workgroup, returned to every thread (fixed shuffle/LDS order).
__device__ inline double block_sum_all(double v) {
  __shared__ double red[kBlock / kWave];
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < kBlock / kWave; ++w) s += red[w];
  return s;
}

__device__ inline double block_max_all(double v) {
  __shared__ double red[kBlock / kWave];
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, kWave));
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < kBlock / kWave; ++w) s = fmax(s, red[w]);
  return s;
}

// Fixed-order sum of part[0..n) by the whole workgroup (same value in every workgroup).
__device__ inline double sum_parts(const double* __restrict__ part, int n) {
  double s = 0.0;
  for (int k = threadIdx.x; k < n; k += kBlock) s += part[k];
  return block_sum_all(s);
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

__global__ void __launch_bounds__(kBlock)
k_spmv(int N, const int* __restrict__ frow_ptr, const int* __restrict__ fcol, const float* __restrict__ fv,
       long long st, const float* __restrict__ p, float* __restrict__ q, double* __restrict__ part_pq,
       const PcgScalars* __restrict__ sc) {
  if (sc->done) return;
  const int lb = xcd_block();
  const int rows_per_block = div_up(div_up(N, gridDim.x), kRowsPerPass) * kRowsPerPass;
  const int r0 = lb * rows_per_block;
  const int r1 = min(N, r0 + rows_per_block);
  const int g = threadIdx.x / kGroup, k = threadIdx.x % kGroup;
  double dot = 0.0;
  for (int rb = r0; rb < r1; rb += kRowsPerPass) {
    const int r = rb + g;
    float a0 = 0.f, a1 = 0.f, a2 = 0.f;
    if (r < r1) {
      const int je = frow_ptr[r + 1];
      for (int j = frow_ptr[r] + k; j < je; j += kGroup) {
        const int c = fcol[j];
        const float pc0 = p[3LL * c], pc1 = p[3LL * c + 1], pc2 = p[3LL * c + 2];
        a0 += fv[j] * pc0 + fv[st + j] * pc1 + fv[2 * st + j] * pc2;
        a1 += fv[3 * st + j] * pc0 + fv[4 * st + j] * pc1 + fv[5 * st + j] * pc2;
        a2 += fv[6 * st + j] * pc0 + fv[7 * st + j] * pc1 + fv[8 * st + j] * pc2;
      }
    }
#pragma unroll
    for (int off = kGroup / 2; off > 0; off >>= 1) {
      a0 += __shfl_xor(a0, off, kGroup);
      a1 += __shfl_xor(a1, off, kGroup);
      a2 += __shfl_xor(a2, off, kGroup);
    }
    if (r < r1 && k == 0) {
      const float pr0 = p[3LL * r], pr1 = p[3LL * r + 1], pr2 = p[3LL * r + 2];
      const float q0 = pr0 + a0, q1 = pr1 + a1, q2 = pr2 + a2;   // identity diagonal block
      q[3LL * r] = q0;
      q[3LL * r + 1] = q1;
      q[3LL * r + 2] = q2;
      dot += (double)pr0 * q0 + (double)pr1 * q1 + (double)pr2 * q2;
    }
  }
  put_part(part_pq, block_sum_all(dot));
}

__global__ void __launch_bounds__(kBlock)
k_update(int N, const float* __restrict__ Lf, float* __restrict__ x, float* __restrict__ r,
         const float* __restrict__ p, const float* __restrict__ q, const double* __restrict__ part_pq, int n_pq,
         double* __restrict__ part_rr, double* __restrict__ part_rt, PcgScalars* __restrict__ sc) {
  if (sc->done) return;
  const int k = sc->iter3;
  const double rho = sum_parts(part_rr + (k & 1) * kGridVec, gridDim.x);
  const double pq = sum_parts(part_pq, n_pq);
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
  for (int v = blockIdx.x * kBlock + threadIdx.x; v < N; v += gridDim.x * kBlock) {
    const long long o = 3LL * v;
    const float r0 = r[o] - alpha * q[o], r1 = r[o + 1] - alpha * q[o + 1], r2 = r[o + 2] - alpha * q[o + 2];
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
  put_part(part_rr + ((k + 1) & 1) * kGridVec, block_sum_all(rr));
  put_part(part_rt, block_sum_all(rt));
}

__global__ void __launch_bounds__(kBlock)
k_direction(int N, const float* __restrict__ r, float* __restrict__ p, const double* __restrict__ part_rr,
            const double* __restrict__ part_rt, PcgScalars* __restrict__ sc) {
  if (sc->done) return;
  const int k = sc->iter2;
  const double rho_old = sum_parts(part_rr + (k & 1) * kGridVec, gridDim.x);
  const double rho_new = sum_parts(part_rr + ((k + 1) & 1) * kGridVec, gridDim.x);
  const bool check = ((k + 1) % sc->check_every) == 0;
  const double rt = check ? sum_parts(part_rt, gridDim.x) : 0.0;
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
  const long long n3 = 3LL * N;
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n3; i += (long long)gridDim.x * kBlock)
    p[i] = r[i] + beta * p[i];
}

__global__ void __launch_bounds__(kBlock)
k_init(int N, const float* __restrict__ bhat, float* __restrict__ x, float* __restrict__ r, float* __restrict__ p,
       double* __restrict__ part_rr) {
  double rr = 0.0;
  const long long n3 = 3LL * N;
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n3; i += (long long)gridDim.x * kBlock) {
    const float b = bhat[i];
    x[i] = 0.f;
    r[i] = b;
    p[i] = b;
    rr += (double)b * b;
  }
  put_part(part_rr, block_sum_all(rr));   // iteration 0 reads slot (0 & 1) = 0
}

__global__ void __launch_bounds__(kBlock)
k_init_scalars(const double* __restrict__ bb_part, int nbb, PcgScalars* sc, double tol, int max_iter,
               int check_every) {
  const double bb = sum_parts(bb_part, nbb);
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
__global__ void __launch_bounds__(kBlock)
k_finish(int N, const float* __restrict__ Linv, const float* __restrict__ x, double* __restrict__ pout,
         double* __restrict__ part) {
  double m = 0.0;
  for (int v = blockIdx.x * kBlock + threadIdx.x; v < N; v += gridDim.x * kBlock) {
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
  const double s = block_max_all(m);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kBlock)
k_finish_scalars(const double* __restrict__ part, int n, const double* __restrict__ viol_part, int nviol,
                 PcgScalars* sc) {
  double m = 0.0, vm = 0.0;
  for (int k = threadIdx.x; k < n; k += kBlock) m = fmax(m, part[k]);
  for (int k = threadIdx.x; k < nviol; k += kBlock) vm = fmax(vm, viol_part[k]);
  m = block_max_all(m);
  vm = block_max_all(vm);
  if (threadIdx.x == 0) {
    sc->stat_pinf = m;
    sc->stat_viol = vm;
  }
}

inline int vec_grid(int N) {
  int g = div_up(N, kBlock);
  return g < 1 ? 1 : (g > kGridVec ? kGridVec : g);
}

inline int spmv_grid(int N) {
  int g = div_up(N, kRowsPerPass);
  if (g > kGridSpmv) g = kGridSpmv;
  return ((g + 7) / 8) * 8;
}

}  // namespace

// Partials layout: [0, 2*kGridVec) r^T r of two consecutive iterations,
// [2k, 3k) |L r|^2, [3k, 3k + kGridSpmv) p^T q  (k = kGridVec).
int pcg_partials_needed(int N) {
  (void)N;
  return 3 * kGridVec + kGridSpmv + 64;
}

void launch_pcg_init(int N, const float* bhat, float* x, float* r, float* p, double* part, const double* bb_part,
                     int nbb, PcgScalars* sc, double tol, int max_iter, int check_every, hipStream_t s) {
  hipLaunchKernelGGL(k_init, dim3(vec_grid(N)), dim3(kBlock), 0, s, N, bhat, x, r, p, part);
  hipLaunchKernelGGL(k_init_scalars, dim3(1), dim3(kBlock), 0, s, bb_part, nbb, sc, tol, max_iter, check_every);
}

void launch_pcg_spmv(int N, const int* frow_ptr, const int* fcol, const float* fvals, long long fstride,
                     const float* p, float* q, double* part, PcgScalars* sc, hipStream_t s) {
  hipLaunchKernelGGL(k_spmv, dim3(spmv_grid(N)), dim3(kBlock), 0, s, N, frow_ptr, fcol, fvals, fstride, p, q,
                     part + 3 * kGridVec, (const PcgScalars*)sc);
}

void launch_pcg_vector_ops(int N, const float* Lf, float* x, float* r, float* p, const float* q, double* part,
                           PcgScalars* sc, hipStream_t s) {
  const int gv = vec_grid(N);
  hipLaunchKernelGGL(k_update, dim3(gv), dim3(kBlock), 0, s, N, Lf, x, r, (const float*)p, q,
                     (const double*)(part + 3 * kGridVec), spmv_grid(N), part, part + 2 * kGridVec, sc);
  hipLaunchKernelGGL(k_direction, dim3(gv), dim3(kBlock), 0, s, N, (const float*)r, p, (const double*)part,
                     (const double*)(part + 2 * kGridVec), sc);
}

void launch_pcg_finish(int N, const float* Linv, const float* x, double* pout, double* part, PcgScalars* sc,
                       const double* viol_part, int nviol, hipStream_t s) {
  const int g = vec_grid(N);
  hipLaunchKernelGGL(k_finish, dim3(g), dim3(kBlock), 0, s, N, Linv, x, pout, part);
  hipLaunchKernelGGL(k_finish_scalars, dim3(1), dim3(kBlock), 0, s, (const double*)part, g, viol_part, nviol, sc);
}

}  // namespace bfal
