// The rest of SolveSubproblem (Algorithm 2) around the Newton step:
//  - the total energy L of Section 4.2 in FP64, with every slack at its
//    minimizer s_i = max(0, c_i - lambda_i/mu) (so L depends on x_hat alone and
//    the step's G is its gradient): 1/2 |x - x_tilde|_M^2 + h^2 sum V_e Psi(F_e)
//    + sum gamma_i (mu/2 (c_i - s_i)^2 - lambda_i (c_i - s_i)), for the line
//    search.  The Neo-Hookean density is the one the element kernel
//    differentiates; a tet with det F <= 0 has no finite energy (the model is
//    non-invertible) and is reported instead.  The element quantities (D_m^-1,
//    V_e, Lame parameters) are rebuilt in FP64 from the rest shape, and the
//    lumped mass rho V_e / 4 is folded per tet, so the whole sum is FP64;
//  - the trial state x_hat + r p;
//  - the multiplier and decay update after the Newton loop: s_i = 0 gives
//    lambda_i -= mu c_i and gamma_i = 1, s_i > 0 gives lambda_i = 0 and
//    gamma_i *= Gamma (Section 4.2, "Constraint Decay");
//  - the conditioning-aware penalty of Section 5.2, C max_i (grad^2 E)_ii: the
//    largest scalar diagonal of the lumped mass plus the SPD-projected elastic
//    Hessian (the matrix the solver assembles), at the start-of-step state.
// Sums use per-workgroup FP64 partials summed in a fixed order.
#include "common.h"

namespace bfal {

namespace {

constexpr int kEBlock = 256;

template <int NT>
__device__ inline double wg_sum(double v) {
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

__device__ inline double det3(const double a[3][3]) {
  return a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1]) - a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0]) +
         a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]);
}

// c_i(x) = d_i + grad d_i^T (x - x_lin) - delta from the FP64 linearization.
__device__ inline double constraint_value(const int4 t, int i, int n_c, const double* __restrict__ lin64,
                                          const double* __restrict__ xlin, const double* __restrict__ x,
                                          double delta) {
  const double d = lin64[i];
  const double n0 = lin64[(long long)n_c + i], n1 = lin64[2LL * n_c + i], n2 = lin64[3LL * n_c + i];
  const int v[4] = {t.x, t.y, t.z, t.w};
  double c = d - delta;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const double w = lin64[(4LL + a) * n_c + i];
    const long long o = 3LL * v[a];
    c += w * (n0 * (x[o] - xlin[o]) + n1 * (x[o + 1] - xlin[o + 1]) + n2 * (x[o + 2] - xlin[o + 2]));
  }
  return c;
}

// Sum over k of S_k - 1 and of (S_k - 1)^2 for the singular values S_k of
// F = I + G (all positive, J > 0), without cancellation near rest: the
// eigenvalues e_k of F^T F - I = G + G^T + G^T G by cyclic Jacobi, then
// S_k - 1 = e_k / (1 + sqrt(1 + e_k)).
__device__ void stretch_sums(const double G[3][3], double& sum1, double& sum2) {
  double A[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      A[i][j] = G[i][j] + G[j][i] + G[0][i] * G[0][j] + G[1][i] * G[1][j] + G[2][i] * G[2][j];
  for (int sweep = 0; sweep < 16; ++sweep) {
    const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    const double dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
    if (off <= 1e-34 * dia || off == 0.0) break;
    for (int pq = 0; pq < 3; ++pq) {
      const int p = pq == 2 ? 1 : 0;
      const int q = pq == 0 ? 1 : 2;
      const double apq = A[p][q];
      if (apq == 0.0) continue;
      const double theta = (A[q][q] - A[p][p]) / (2.0 * apq);
      const double t = copysign(1.0, theta) / (fabs(theta) + sqrt(theta * theta + 1.0));
      const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
      const int r = 3 - p - q;
      const double arp = A[r][p], arq = A[r][q];
      A[p][p] -= t * apq;
      A[q][q] += t * apq;
      A[p][q] = A[q][p] = 0.0;
      A[r][p] = A[p][r] = c * arp - s * arq;
      A[r][q] = A[q][r] = s * arp + c * arq;
    }
  }
  sum1 = sum2 = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double d = A[k][k] / (1.0 + sqrt(fmax(1.0 + A[k][k], 0.0)));
    sum1 += d;
    sum2 += d * d;
  }
}

// One partial per workgroup: tets in the first ceil(T / kEBlock) workgroups,
// constraints in the next ceil(n_c / kEBlock), friction contacts in the rest.
__global__ void __launch_bounds__(kEBlock)
k_energy(const int4* __restrict__ tets, int T, const double* __restrict__ rest, const double* __restrict__ E,
         const double* __restrict__ nu, const double* __restrict__ rho, double h2, const double* __restrict__ x,
         const double* __restrict__ xt, const int4* __restrict__ ids, int n_c, const double* __restrict__ lin64,
         const double* __restrict__ xlin, const double* __restrict__ lam, const double* __restrict__ gam,
         double kappa, double delta, int tet_groups, int con_groups, const int* __restrict__ mat, FrictionView fr,
         double* __restrict__ part, int* inverted) {
  double e = 0.0;
  if ((int)blockIdx.x < tet_groups) {
    const int k = blockIdx.x * kEBlock + threadIdx.x;
    if (k < T) {
      const int4 t = tets[k];
      const int v[4] = {t.x, t.y, t.z, t.w};
      double Dm[3][3], Ds[3][3];
#pragma unroll
      for (int a = 1; a < 4; ++a)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          Dm[i][a - 1] = rest[3LL * v[a] + i] - rest[3LL * v[0] + i];
          Ds[i][a - 1] = x[3LL * v[a] + i] - x[3LL * v[0] + i];
        }
      const double dm = det3(Dm);
      const double vol = fabs(dm) / 6.0;
      // D_m^{-1} by cofactors
      double Di[3][3];
      Di[0][0] = (Dm[1][1] * Dm[2][2] - Dm[1][2] * Dm[2][1]) / dm;
      Di[0][1] = (Dm[0][2] * Dm[2][1] - Dm[0][1] * Dm[2][2]) / dm;
      Di[0][2] = (Dm[0][1] * Dm[1][2] - Dm[0][2] * Dm[1][1]) / dm;
      Di[1][0] = (Dm[1][2] * Dm[2][0] - Dm[1][0] * Dm[2][2]) / dm;
      Di[1][1] = (Dm[0][0] * Dm[2][2] - Dm[0][2] * Dm[2][0]) / dm;
      Di[1][2] = (Dm[0][2] * Dm[1][0] - Dm[0][0] * Dm[1][2]) / dm;
      Di[2][0] = (Dm[1][0] * Dm[2][1] - Dm[1][1] * Dm[2][0]) / dm;
      Di[2][1] = (Dm[0][1] * Dm[2][0] - Dm[0][0] * Dm[2][1]) / dm;
      Di[2][2] = (Dm[0][0] * Dm[1][1] - Dm[0][1] * Dm[1][0]) / dm;
      double F[3][3];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) F[i][j] = Ds[i][0] * Di[0][j] + Ds[i][1] * Di[1][j] + Ds[i][2] * Di[2][j];
      const double J = det3(F);
      const double Ey = E[k], ny = nu[k];
      const double mu = Ey / (2.0 * (1.0 + ny));
      const double la = Ey * ny / ((1.0 + ny) * (1.0 - 2.0 * ny));
      if (!(J > 0.0)) {
        atomicOr(inverted, 1);
      } else {
        double I1 = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) I1 += F[i][j] * F[i][j];
        double psi;
        const int code = mat != nullptr ? mat[k] : 0;
        if (code == 2) {
          // corotated linear: mu sum (S_i - 1)^2 + lam/2 (sum S_i - 3)^2
          double G[3][3], s1, s2;
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) G[i][j] = F[i][j] - (i == j ? 1.0 : 0.0);
          stretch_sums(G, s1, s2);
          psi = mu * s2 + 0.5 * la * s1 * s1;
        } else if (code == 1) {
          psi = 0.5 * mu * (I1 - 3.0) - mu * (J - 1.0) + 0.5 * la * (J - 1.0) * (J - 1.0);
        } else {
          const double lnJ = log(J);
          psi = 0.5 * mu * (I1 - 3.0) - mu * lnJ + 0.5 * la * lnJ * lnJ;
        }
        e = h2 * vol * psi;
      }
      // inertia: the lumped mass rho V / 4 of each vertex, folded per tet
      double in = 0.0;
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          const double dd = x[3LL * v[a] + i] - xt[3LL * v[a] + i];
          in += dd * dd;
        }
      e += 0.5 * (rho[k] * vol / 4.0) * in;
    }
  } else if ((int)blockIdx.x >= tet_groups + con_groups) {
    // friction (Appendix A): coef f_0(|u|) with IPC's smoothed norm, e = eps_v h
    const int i = (blockIdx.x - tet_groups - con_groups) * kEBlock + threadIdx.x;
    if (i < fr.n_f) {
      const int4 t = fr.ids[i];
      const int vv[4] = {t.x, t.y, t.z, t.w};
      const long long nf = fr.n_f;
      double v[3] = {0.0, 0.0, 0.0};
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const double wa = fr.f64[(3 + a) * nf + i];
#pragma unroll
        for (int k = 0; k < 3; ++k) v[k] += wa * (x[3LL * vv[a] + k] - fr.x0[3LL * vv[a] + k]);
      }
      const double n0 = fr.f64[i], n1 = fr.f64[nf + i], n2 = fr.f64[2 * nf + i];
      const double vn = n0 * v[0] + n1 * v[1] + n2 * v[2];
      const double u0 = v[0] - vn * n0, u1 = v[1] - vn * n1, u2 = v[2] - vn * n2;
      const double y = sqrt(u0 * u0 + u1 * u1 + u2 * u2), ee = fr.e;
      const double f0 = y >= ee ? y : -y * y * y / (3.0 * ee * ee) + y * y / ee + ee / 3.0;
      e = fr.f64[7 * nf + i] * f0;
    }
  } else {
    const int i = (blockIdx.x - tet_groups) * kEBlock + threadIdx.x;
    if (i < n_c) {
      const double c = constraint_value(ids[i], i, n_c, lin64, xlin, x, delta);
      const double l = lam[i], g = gam[i];
      const double cs = c - fmax(0.0, c - l / kappa);   // c - s at the minimizing slack
      e = g * (0.5 * kappa * cs * cs - l * cs);
    }
  }
  const double s = wg_sum<kEBlock>(e);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kEBlock)
k_state_axpy(int n3, const double* __restrict__ xa, double r, const double* __restrict__ p, double* __restrict__ xt) {
  const int i = blockIdx.x * kEBlock + threadIdx.x;
  if (i < n3) xt[i] = xa[i] + r * p[i];
}

// Partials per workgroup: [0, g) active counts, [g, 2g) max violation.
__global__ void __launch_bounds__(kEBlock)
k_dual_update(const int4* __restrict__ ids, int n_c, const double* __restrict__ lin64,
              const double* __restrict__ xlin, const double* __restrict__ xh, double kappa, double delta,
              double decay, double* __restrict__ lam, double* __restrict__ gam, double* __restrict__ part) {
  const int i = blockIdx.x * kEBlock + threadIdx.x;
  double act = 0.0, viol = 0.0;
  if (i < n_c) {
    const double c = constraint_value(ids[i], i, n_c, lin64, xlin, xh, delta);
    const double l = lam[i];
    const double s = fmax(0.0, c - l / kappa);
    if (s == 0.0) {
      lam[i] = l - kappa * c;
      gam[i] = 1.0;
      act = 1.0;
    } else {
      lam[i] = 0.0;
      gam[i] = decay * gam[i];
    }
    viol = fmax(0.0, -c);
  }
  const double sa = wg_sum<kEBlock>(act);
  // block max of the violation
  __shared__ double red[kEBlock / kWave];
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) viol = fmax(viol, __shfl_xor(viol, off, kWave));
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = viol;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = red[0];
    for (int w = 1; w < kEBlock / kWave; ++w) m = fmax(m, red[w]);
    part[blockIdx.x] = sa;
    part[gridDim.x + blockIdx.x] = m;
  }
}

// Largest scalar diagonal of M + h^2 (projected elastic Hessian), per
// workgroup: the diagonal block of row r is the sum of its staging range (the
// static pattern holds the diagonal first in each row), plus the lumped mass.
__global__ void __launch_bounds__(kEBlock)
k_diag_max(int N, const int* __restrict__ erow_ptr, const int* __restrict__ ecptr, const double* __restrict__ staging,
           const double* __restrict__ mass, double* __restrict__ part) {
  const int r = blockIdx.x * kEBlock + threadIdx.x;
  double m = 0.0;
  if (r < N) {
    const int es = erow_ptr[r];
    double d0 = 0.0, d1 = 0.0, d2 = 0.0;
    for (int j = ecptr[es]; j < ecptr[es + 1]; ++j) {
      const double* st = staging + 9LL * j;   // symmetric 6 (xx, xy, xz, yy, yz, zz), then the gradient
      d0 += st[0];
      d1 += st[3];
      d2 += st[5];
    }
    const double mv = mass[r];
    m = fmax(fmax(d0 + mv, d1 + mv), d2 + mv);
  }
  __shared__ double red[kEBlock / kWave];
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, kWave));
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = red[0];
    for (int w = 1; w < kEBlock / kWave; ++w) b = fmax(b, red[w]);
    part[blockIdx.x] = b;
  }
}

// x += alpha (x_hat - x): the next intersection-free state (Algorithm 1).
__global__ void __launch_bounds__(kEBlock)
k_blend(int n3, double* __restrict__ x, const double* __restrict__ xh, double alpha) {
  const int i = blockIdx.x * kEBlock + threadIdx.x;
  if (i < n3) x[i] = (1.0 - alpha) * x[i] + alpha * xh[i];
}

__global__ void __launch_bounds__(kEBlock)
k_velocity(int n3, const double* __restrict__ x, const double* __restrict__ x0, double inv_h, double* __restrict__ v) {
  const int i = blockIdx.x * kEBlock + threadIdx.x;
  if (i < n3) v[i] = (x[i] - x0[i]) * inv_h;
}

}  // namespace

void launch_blend(int n3, double* x, const double* xh, double alpha, hipStream_t s) {
  hipLaunchKernelGGL(k_blend, dim3(div_up(n3, kEBlock)), dim3(kEBlock), 0, s, n3, x, xh, alpha);
}

void launch_velocity(int n3, const double* x, const double* x0, double inv_h, double* v, hipStream_t s) {
  hipLaunchKernelGGL(k_velocity, dim3(div_up(n3, kEBlock)), dim3(kEBlock), 0, s, n3, x, x0, inv_h, v);
}

int energy_parts(int T, int n_c, int n_f) { return div_up(T, kEBlock) + div_up(n_c, kEBlock) + div_up(n_f, kEBlock); }

int diag_max_parts(int N) { return div_up(N, kEBlock); }

void launch_diag_max(int N, const int* erow_ptr, const int* ecptr, const double* staging, const double* mass,
                     double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_diag_max, dim3(div_up(N, kEBlock)), dim3(kEBlock), 0, s, N, erow_ptr, ecptr, staging, mass,
                     part);
}

void launch_energy(const int4* tets, int T, const double* rest, const double* E, const double* nu,
                   const double* rho, double h, const double* x, const double* xt, const int4* ids, int n_c,
                   const double* lin64, const double* xlin, const double* lam, const double* gam, double kappa,
                   double delta, const int* mat, FrictionView fr, double* part, int* inverted, hipStream_t s) {
  const int tg = div_up(T, kEBlock), cg = div_up(n_c, kEBlock);
  const int g = energy_parts(T, n_c, fr.n_f);
  hipLaunchKernelGGL(k_energy, dim3(g), dim3(kEBlock), 0, s, tets, T, rest, E, nu, rho, h * h, x, xt, ids, n_c, lin64,
                     xlin, lam, gam, kappa, delta, tg, cg, mat, fr, part, inverted);
}

void launch_state_axpy(int n3, const double* xa, double r, const double* p, double* xt, hipStream_t s) {
  hipLaunchKernelGGL(k_state_axpy, dim3(div_up(n3, kEBlock)), dim3(kEBlock), 0, s, n3, xa, r, p, xt);
}

void launch_dual_update(const int4* ids, int n_c, const double* lin64, const double* xlin, const double* xh,
                        double kappa, double delta, double decay, double* lam, double* gam, double* part,
                        hipStream_t s) {
  if (n_c > 0)
    hipLaunchKernelGGL(k_dual_update, dim3(div_up(n_c, kEBlock)), dim3(kEBlock), 0, s, ids, n_c, lin64, xlin, xh,
                       kappa, delta, decay, lam, gam, part);
}

}  // namespace bfal
