// Hyperelastic element kernel (Neo-Hookean, stable Neo-Hookean or corotated
// linear per tet): one thread per tet.
//
// Per tet it forms, all in FP64, G = F - I and the stress P (from the FP64
// displacement differences and the FP64 rows of D_m^{-1}), the element
// gradient h^2 V P A_a^T, and the ten upper 3x3 blocks of the SPD-projected
// element Hessian by the vertex-block identity of Section 5.1:
//
//   H_ab = h^2 V  U [ sum_k omega_k^+ D_k (A_a V)^T (A_b V) D_k^T ] U^T
//
// where F = U Sigma V^T is a rotation-preserving SVD and (omega_k, D_k) are
// the analytic eigenpairs of d2Psi/dF2 in the SVD frame: three scaling modes
// (eigenvectors e_k of the 3x3 Hessian of Psi in the singular values, D_k =
// diag(e_k)), three twist and three flip modes (D = (E_ij -+ E_ji)/sqrt 2).
// Exploiting the sparsity of D_k, the bracket is the Hadamard product of the
// projected 3x3 scaling Hessian with (A_a V)^T (A_b V), plus four terms per
// singular-value pair.  Blocks are written in FP64 to the fixed assembly
// order (staging position of each (tet, pair)), so no atomics touch the
// matrix.  The Hessian is FP64 because the blocks of one element sum to zero
// along every row and column (A_0 = -(A_1 + A_2 + A_3)): the assembled
// matrix leaves rigid translations to inertia and contact alone, and
// rounding each element's blocks to FP32 breaks that cancellation by about
// 1e-7 of the element stiffness, which on a stiff, finely meshed scene is a
// large relative error in those soft directions.  The row sums assemble the
// FP64 blocks and round the finished matrix once.
//
// Energies (readings of the paper, which names its materials in Table 2
// without printing them); the first two are Psi = mu/2 (tr F^T F - 3) + g(J):
//   Neo-Hookean         g = -mu ln J + lam/2 (ln J)^2
//   stable Neo-Hookean  g = -mu (J - 1) + lam/2 (J - 1)^2   (rest-stable form of
//                       Smith, de Goes and Kim 2019)
// The stress is formed in FP64 because the strain can be far smaller than G:
// a tet turned by a rotation R has G ~ R - I of order one while F^T F - I is
// of the order of its strain, and in FP32 that difference keeps only
// eps / strain of relative accuracy (1e-4 at a 1e-3 strain).  With G = F - I,
//   J - 1 = tr G + ((tr G)^2 - tr(G^2))/2 + det G,  ln J = log1p(J - 1),
//   Neo-Hookean  P = F^{-T} [ mu (G + G^T + G^T G) + lam ln J I ],
//   stable NH    P = mu (G + G^T - tr(G) I - cof G) + lam (J - 1) cof F
// (the second from cof(I + G) = (1 + tr G) I - G^T + cof G); these forms
// are free of cancellation near rest as well.
// With q = J g'(J) and r = J^2 g''(J) the Hessian of Psi in the singular
// values is mu I + diag(r / S_i^2) off-diagonal (r + q) / (S_i S_j), and the
// twist / flip eigenvalues of pair (i, j) are mu +- q / (S_i S_j):
//   Neo-Hookean  q = lam ln J - mu,          r = mu + lam - lam ln J
//   stable NH    q = J (lam (J - 1) - mu),  r = lam J^2.
// Corotated linear (Table 2's COR, F = R S the polar decomposition):
//   Psi = mu ||F - R||^2 + lam/2 (tr S - 3)^2 = mu sum (S_k - 1)^2 + lam/2 (sum S_k - 3)^2,
// whose Hessian in the singular values is 2 mu I + lam 1 1^T and whose twist /
// flip eigenvalues are (Psi_i + Psi_j) / (S_i + S_j) and 2 mu.
#include "common.h"

namespace bfal {

namespace {

__constant__ int c_pa[10] = {0, 0, 0, 0, 1, 1, 1, 2, 2, 3};
__constant__ int c_pb[10] = {0, 1, 2, 3, 1, 2, 3, 2, 3, 3};

// Cyclic Jacobi eigen-decomposition of a symmetric 3x3 matrix (A is destroyed).
// On return A's diagonal holds the eigenvalues and V's columns the eigenvectors.
__device__ inline void jacobi3(double A[3][3], double V[3][3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) V[i][j] = (i == j) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 10; ++sweep) {
    const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    const double dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
    if (off <= 1e-32 * dia || off == 0.0) break;
#pragma unroll
    for (int pq = 0; pq < 3; ++pq) {
      const int p = pq == 2 ? 1 : 0;
      const int q = pq == 0 ? 1 : 2;
      const double apq = A[p][q];
      if (apq == 0.0) continue;
      const double theta = (A[q][q] - A[p][p]) / (2.0 * apq);
      const double t = copysign(1.0, theta) / (fabs(theta) + sqrt(theta * theta + 1.0));
      const double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
      const int r = 3 - p - q;
      const double arp = A[r][p], arq = A[r][q];
      A[p][p] -= t * apq;
      A[q][q] += t * apq;
      A[p][q] = A[q][p] = 0.0;
      A[r][p] = A[p][r] = c * arp - sn * arq;
      A[r][q] = A[q][r] = sn * arp + c * arq;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double vkp = V[k][p], vkq = V[k][q];
        V[k][p] = c * vkp - sn * vkq;
        V[k][q] = sn * vkp + c * vkq;
      }
    }
  }
}

__device__ inline double det3d(const double M[3][3]) {
  return M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
         M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
}

__device__ inline void cof3d(const double M[3][3], double C[3][3]) {
  C[0][0] = M[1][1] * M[2][2] - M[1][2] * M[2][1];
  C[0][1] = M[1][2] * M[2][0] - M[1][0] * M[2][2];
  C[0][2] = M[1][0] * M[2][1] - M[1][1] * M[2][0];
  C[1][0] = M[0][2] * M[2][1] - M[0][1] * M[2][2];
  C[1][1] = M[0][0] * M[2][2] - M[0][2] * M[2][0];
  C[1][2] = M[0][1] * M[2][0] - M[0][0] * M[2][1];
  C[2][0] = M[0][1] * M[1][2] - M[0][2] * M[1][1];
  C[2][1] = M[0][2] * M[1][0] - M[0][0] * M[1][2];
  C[2][2] = M[0][0] * M[1][1] - M[0][1] * M[1][0];
}

// Rotation-preserving SVD F = U diag(S) V^T with det U = det V = +1 (S[2]
// carries the sign of det F).  V from the Jacobi eigenvectors of F^T F, U and
// S from a Givens QR of F V (McAdams et al. 2011, "Computing the singular
// value decomposition of 3x3 matrices with minimal branching and elementary
// floating point operations", steps: symmetric eigenanalysis, sorting, QR).
__device__ inline void svd3(const double F[3][3], double U[3][3], double S[3], double V[3][3]) {
  double A[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) A[i][j] = F[0][i] * F[0][j] + F[1][i] * F[1][j] + F[2][i] * F[2][j];
  double W[3][3];
  jacobi3(A, W);
  const double ev[3] = {A[0][0], A[1][1], A[2][2]};
  int o[3] = {0, 1, 2};
  // sort eigenvalues descending
  if (ev[o[0]] < ev[o[1]]) { int t = o[0]; o[0] = o[1]; o[1] = t; }
  if (ev[o[1]] < ev[o[2]]) { int t = o[1]; o[1] = o[2]; o[2] = t; }
  if (ev[o[0]] < ev[o[1]]) { int t = o[0]; o[0] = o[1]; o[1] = t; }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) V[i][k] = W[i][o[k]];
  if (det3d(V) < 0.0) {
#pragma unroll
    for (int i = 0; i < 3; ++i) V[i][2] = -V[i][2];
  }
  double B[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) B[i][k] = F[i][0] * V[0][k] + F[i][1] * V[1][k] + F[i][2] * V[2][k];
  // Q^T accumulates the Givens rotations: Q^T B = R
  double Qt[3][3] = {{1.0, 0.0, 0.0}, {0.0, 1.0, 0.0}, {0.0, 0.0, 1.0}};
  const int gi[3] = {0, 0, 1}, gj[3] = {1, 2, 2}, gc[3] = {0, 0, 1};
#pragma unroll
  for (int g = 0; g < 3; ++g) {
    const int i = gi[g], j = gj[g], col = gc[g];
    const double a = B[i][col], b = B[j][col];
    const double r = sqrt(a * a + b * b);
    double c = 1.0, sn = 0.0;
    if (r > 0.0) { c = a / r; sn = b / r; }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double bi = B[i][k], bj = B[j][k];
      B[i][k] = c * bi + sn * bj;
      B[j][k] = -sn * bi + c * bj;
      const double qi = Qt[i][k], qj = Qt[j][k];
      Qt[i][k] = c * qi + sn * qj;
      Qt[j][k] = -sn * qi + c * qj;
    }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) U[i][k] = Qt[k][i];
  S[0] = B[0][0]; S[1] = B[1][1]; S[2] = B[2][2];
  // make S[0], S[1] non-negative, pushing signs into column 2 to keep det U = +1
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    if (S[k] < 0.0) {
      S[k] = -S[k]; S[2] = -S[2];
#pragma unroll
      for (int i = 0; i < 3; ++i) { U[i][k] = -U[i][k]; U[i][2] = -U[i][2]; }
    }
  }
}

__global__ void __launch_bounds__(kBlock)
k_elastic(const int4* __restrict__ tets, int T, const double* __restrict__ rest, const double* __restrict__ xh,
          const double* __restrict__ Dminv9, const float* __restrict__ vol, const float* __restrict__ mu_,
          const float* __restrict__ lam_, double h2, const int* __restrict__ epos, double* __restrict__ staging,
          const int* __restrict__ mat, int* flags) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= T) return;
  const int4 t = tets[e];
  const int v[4] = {t.x, t.y, t.z, t.w};
  // G = F - I from the displacement differences and the rows of D_m^{-1}
  double u0[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) u0[i] = xh[3LL * v[0] + i] - rest[3LL * v[0] + i];
  double Du[3][3];  // column k = u_{k+1} - u_0
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int i = 0; i < 3; ++i) Du[i][k] = (xh[3LL * v[k + 1] + i] - rest[3LL * v[k + 1] + i]) - u0[i];
  double Dm[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) Dm[i][j] = Dminv9[(long long)(3 * i + j) * T + e];
  double Gd[3][3], F[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      Gd[i][j] = Du[i][0] * Dm[0][j] + Du[i][1] * Dm[1][j] + Du[i][2] * Dm[2][j];
      F[i][j] = Gd[i][j] + (i == j ? 1.0 : 0.0);
    }
  // C - I = G + G^T + G^T G (the strain)
  double CmI[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      CmI[i][j] = Gd[i][j] + Gd[j][i] + Gd[0][i] * Gd[0][j] + Gd[1][i] * Gd[1][j] + Gd[2][i] * Gd[2][j];
  const double trG = Gd[0][0] + Gd[1][1] + Gd[2][2];
  double trG2 = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) trG2 += Gd[i][j] * Gd[j][i];
  const double Jm1 = trG + 0.5 * (trG * trG - trG2) + det3d(Gd);
  const double J = 1.0 + Jm1;
  const double w = h2 * (double)vol[e];
  const long long pbase = 10LL * e;
  if (!(J > 0.0)) {
    atomicOr(flags, FLAG_INVERTED);
    for (int k = 0; k < 10; ++k) {
      double* o = staging + 9LL * epos[pbase + k];
#pragma unroll
      for (int q = 0; q < 9; ++q) o[q] = 0.0;
    }
    return;
  }
  const double mu = mu_[e], lam = lam_[e];
  const int code = mat != nullptr ? mat[e] : 0;
  // rows A_a (A_1..A_3 = rows of Dm^{-1}, A_0 = -their sum)
  double A[4][3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    A[1][j] = Dm[0][j]; A[2][j] = Dm[1][j]; A[3][j] = Dm[2][j];
    A[0][j] = -(Dm[0][j] + Dm[1][j] + Dm[2][j]);
  }
  // SVD, then per material the stress, the 3x3 Hessian in the singular values
  // (Ah) and the twist / flip eigenvalues of the pairs (0,1), (0,2), (1,2)
  double U[3][3], S[3], V[3][3];
  svd3(F, U, S, V);
  const int pi[3] = {0, 0, 1}, pj[3] = {1, 2, 2};
  double P[3][3], Ah[3][3], wt[3], wf[3];
  bool clamp;
  if (code == 2) {
    // corotated linear: Psi = mu sum (S_k - 1)^2 + lam/2 (sum S_k - 3)^2.  S_k - 1 without
    // cancellation: e_k = S_k^2 - 1 is the Rayleigh quotient of F^T F - I along V_k
    // (stationary in V_k), and S_k - 1 = e_k / (1 + sqrt(1 + e_k)).
    double d[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double ek = 0.0;
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) ek += V[i][k] * CmI[i][j] * V[j][k];
      d[k] = ek / (1.0 + sqrt(fmax(1.0 + ek, 0.0)));
    }
    const double tr = d[0] + d[1] + d[2];
    double dpsi[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) dpsi[k] = 2.0 * mu * d[k] + lam * tr;
    // P = U diag(dPsi/dS) V^T = 2 mu (F - R) + lam tr(S - I) R
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        P[i][j] = U[i][0] * dpsi[0] * V[j][0] + U[i][1] * dpsi[1] * V[j][1] + U[i][2] * dpsi[2] * V[j][2];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) Ah[i][j] = (i == j ? 2.0 * mu : 0.0) + lam;
    clamp = lam < 0.0;   // 2 mu I + lam 1 1^T is PSD for lam >= 0
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int i = pi[k], j = pj[k];
      wt[k] = (dpsi[i] + dpsi[j]) / (2.0 + d[i] + d[j]);
      wf[k] = 2.0 * mu;   // (dPsi_i - dPsi_j) / (S_i - S_j)
    }
  } else {
    double C[3][3];
    cof3d(F, C);
    double q, r, rq;
    if (code == 1) {
      double Cg[3][3];
      cof3d(Gd, Cg);
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
          P[i][j] = mu * (Gd[i][j] + Gd[j][i] - (i == j ? trG : 0.0) - Cg[i][j]) + lam * Jm1 * C[i][j];
      q = J * (lam * Jm1 - mu);
      r = lam * J * J;
      rq = r + q;
    } else {
      const double lnJ = log1p(Jm1);
      // P = F^{-T} Sp with Sp = mu (C - I) + lam lnJ I; F^{-T} = cof(F) / J
      double Sp[3][3];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) Sp[i][j] = mu * CmI[i][j] + (i == j ? lam * lnJ : 0.0);
      const double iJ = 1.0 / J;
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) P[i][j] = (C[i][0] * Sp[0][j] + C[i][1] * Sp[1][j] + C[i][2] * Sp[2][j]) * iJ;
      q = lam * lnJ - mu;
      r = mu + lam - lam * lnJ;
      rq = lam;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) Ah[i][j] = (i == j) ? mu + r / (S[i] * S[i]) : rq / (S[i] * S[j]);
    // Ah = mu I + diag(1/S) (-q I + (r + q) 1 1^T) diag(1/S) is PSD when -q >= 0 and r + q >= 0
    clamp = q > 0.0 || rq < 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double ss = S[pi[k]] * S[pj[k]];
      wt[k] = mu + q / ss;
      wf[k] = mu - q / ss;
    }
  }
  if (clamp) {
    // Ah may be indefinite: clamp its eigenvalues
    double E3[3][3], Q[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) E3[i][j] = Ah[i][j];
    jacobi3(E3, Q);
    const double l0 = fmax(E3[0][0], 0.0), l1 = fmax(E3[1][1], 0.0), l2 = fmax(E3[2][2], 0.0);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) Ah[i][j] = l0 * Q[i][0] * Q[j][0] + l1 * Q[i][1] * Q[j][1] + l2 * Q[i][2] * Q[j][2];
  }
  double c1[3], c2[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double tk = fmax(wt[k], 0.0), fk = fmax(wf[k], 0.0);
    c1[k] = 0.5 * (tk + fk);
    c2[k] = 0.5 * (fk - tk);
  }
  double AV[4][3];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int k = 0; k < 3; ++k) AV[a][k] = A[a][0] * V[0][k] + A[a][1] * V[1][k] + A[a][2] * V[2][k];

  for (int pr = 0; pr < 10; ++pr) {
    const int a = c_pa[pr], b = c_pb[pr];
    double Sm[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) Sm[i][j] = Ah[i][j] * AV[a][i] * AV[b][j];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int i = pi[k], j = pj[k];
      Sm[i][i] += c1[k] * AV[a][j] * AV[b][j];
      Sm[j][j] += c1[k] * AV[a][i] * AV[b][i];
      Sm[i][j] += c2[k] * AV[a][j] * AV[b][i];
      Sm[j][i] += c2[k] * AV[a][i] * AV[b][j];
    }
    double T1[3][3], Hb[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) T1[i][j] = U[i][0] * Sm[0][j] + U[i][1] * Sm[1][j] + U[i][2] * Sm[2][j];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) Hb[i][j] = w * (T1[i][0] * U[j][0] + T1[i][1] * U[j][1] + T1[i][2] * U[j][2]);
    double* o = staging + 9LL * epos[pbase + pr];
    if (a == b) {
      // symmetric diagonal block: 6 entries, then the vertex gradient h^2 V P A_a^T
      o[0] = Hb[0][0];
      o[1] = 0.5 * (Hb[0][1] + Hb[1][0]);
      o[2] = 0.5 * (Hb[0][2] + Hb[2][0]);
      o[3] = Hb[1][1];
      o[4] = 0.5 * (Hb[1][2] + Hb[2][1]);
      o[5] = Hb[2][2];
#pragma unroll
      for (int i = 0; i < 3; ++i) o[6 + i] = w * (P[i][0] * A[a][0] + P[i][1] * A[a][1] + P[i][2] * A[a][2]);
    } else if (v[a] < v[b]) {
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) o[3 * i + j] = Hb[i][j];
    } else {
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) o[3 * i + j] = Hb[j][i];
    }
  }
}

}  // namespace

void launch_elastic(const int4* tets, int T, const double* rest, const double* xh, const double* Dminv9,
                    const float* vol, const float* mu, const float* lam, double h2, const int* epos, double* staging,
                    const int* mat, int* flags, hipStream_t s) {
  if (T > 0)
    hipLaunchKernelGGL(k_elastic, dim3(div_up(T, kBlock)), dim3(kBlock), 0, s, tets, T, rest, xh, Dminv9, vol, mu,
                       lam, h2, epos, staging, mat, flags);
}

}  // namespace bfal
