// Per-mesh setup kernels: rest geometry (the constant row vectors A_a that map
// vertex displacements to dF, Section 5.1), Lame parameters, lumped mass
// (Section 3), the static elastic upper 3x3-block pattern, and the fixed
// order in which per-tet blocks are summed into each slot (deterministic,
// atomic-free assembly).
#include "common.h"

namespace bfal {

namespace {

// local vertex pairs of a 4-vertex stencil: the 10 upper blocks, diagonal first
__constant__ int c_pa[10] = {0, 0, 0, 0, 1, 1, 1, 2, 2, 3};
__constant__ int c_pb[10] = {0, 1, 2, 3, 1, 2, 3, 2, 3, 3};

__device__ inline int vtx(const int4& t, int a) { return a == 0 ? t.x : a == 1 ? t.y : a == 2 ? t.z : t.w; }

__global__ void k_check_tets(const int4* __restrict__ tets, int T, int N, int* flags) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= T) return;
  const int4 t = tets[e];
  bool bad = t.x < 0 || t.y < 0 || t.z < 0 || t.w < 0 || t.x >= N || t.y >= N || t.z >= N || t.w >= N ||
             t.x == t.y || t.x == t.z || t.x == t.w || t.y == t.z || t.y == t.w || t.z == t.w;
  if (bad) atomicOr(flags, FLAG_BAD_INDEX);
}

__global__ void k_rest_geometry(const int4* __restrict__ tets, const double* __restrict__ rest,
                                const double* __restrict__ E, const double* __restrict__ nu,
                                const double* __restrict__ rho, int T,
                                double* __restrict__ Dminv9, float* __restrict__ vol,
                                float* __restrict__ mu, float* __restrict__ lam, int* flags) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= T) return;
  const int4 t = tets[e];
  const int v[4] = {t.x, t.y, t.z, t.w};
  double X[4][3];
  for (int a = 0; a < 4; ++a)
    for (int i = 0; i < 3; ++i) X[a][i] = rest[3 * (long long)v[a] + i];
  double D[3][3];  // columns X_k - X_0
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) D[i][k] = X[k + 1][i] - X[0][i];
  const double c00 = D[1][1] * D[2][2] - D[1][2] * D[2][1];
  const double c01 = D[1][2] * D[2][0] - D[1][0] * D[2][2];
  const double c02 = D[1][0] * D[2][1] - D[1][1] * D[2][0];
  const double det = D[0][0] * c00 + D[0][1] * c01 + D[0][2] * c02;
  double scale = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) scale = fmax(scale, fabs(D[i][k]));
  const double En = E[e], nn = nu[e], rh = rho[e];
  if (!(fabs(det) > 1e-12 * scale * scale * scale) || !(En > 0.0 && En < INFINITY) || !(nn > -1.0 && nn < 0.5) ||
      !(rh > 0.0 && rh < INFINITY)) {
    atomicOr(flags, FLAG_BAD_VALUE);
    return;
  }
  const double id = 1.0 / det;
  double inv[3][3];
  inv[0][0] = c00 * id;
  inv[1][0] = c01 * id;
  inv[2][0] = c02 * id;
  inv[0][1] = (D[0][2] * D[2][1] - D[0][1] * D[2][2]) * id;
  inv[1][1] = (D[0][0] * D[2][2] - D[0][2] * D[2][0]) * id;
  inv[2][1] = (D[0][1] * D[2][0] - D[0][0] * D[2][1]) * id;
  inv[0][2] = (D[0][1] * D[1][2] - D[0][2] * D[1][1]) * id;
  inv[1][2] = (D[0][2] * D[1][0] - D[0][0] * D[1][2]) * id;
  inv[2][2] = (D[0][0] * D[1][1] - D[0][1] * D[1][0]) * id;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Dminv9[(long long)(3 * i + j) * T + e] = inv[i][j];
  vol[e] = (float)(fabs(det) / 6.0);
  mu[e] = (float)(En / (2.0 * (1.0 + nn)));
  lam[e] = (float)(En * nn / ((1.0 + nn) * (1.0 - 2.0 * nn)));
}

__global__ void k_pair_count(const int4* __restrict__ tets, int T, int* cnt) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= T) return;
  const int4 t = tets[e];
  for (int k = 0; k < 10; ++k) {
    const int a = c_pa[k], b = c_pb[k];
    if (a == b) continue;
    const int va = vtx(t, a), vb = vtx(t, b);
    atomicAdd(&cnt[min(va, vb)], 1);
  }
}

__global__ void k_pair_fill(const int4* __restrict__ tets, int T, const int* __restrict__ ptr, int* cursor,
                            int* keys) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= T) return;
  const int4 t = tets[e];
  for (int k = 0; k < 10; ++k) {
    const int a = c_pa[k], b = c_pb[k];
    if (a == b) continue;
    const int va = vtx(t, a), vb = vtx(t, b);
    const int lo = min(va, vb), hi = max(va, vb);
    keys[ptr[lo] + atomicAdd(&cursor[lo], 1)] = hi;
  }
}

// Sort a row's keys, drop duplicates in place; ucount = 1 (diagonal) + #unique.
__global__ void k_row_unique(int* keys, const int* __restrict__ kptr, int N, int* ucount) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= N) return;
  const int b = kptr[r], e = kptr[r + 1];
  for (int j = b + 1; j < e; ++j) {
    int key = keys[j];
    int k = j - 1;
    while (k >= b && keys[k] > key) { keys[k + 1] = keys[k]; --k; }
    keys[k + 1] = key;
  }
  int u = 0;
  for (int j = b; j < e; ++j)
    if (j == b || keys[j] != keys[j - 1]) keys[b + u++] = keys[j];
  ucount[r] = 1 + u;
}

__global__ void k_row_write(const int* __restrict__ keys, const int* __restrict__ kptr, int N,
                            const int* __restrict__ row_ptr, int* col) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= N) return;
  const int o = row_ptr[r], n = row_ptr[r + 1] - o;
  col[o] = r;
  const int b = kptr[r];
  for (int j = 1; j < n; ++j) col[o + j] = keys[b + j - 1];
}

__device__ inline int find_slot(const int* __restrict__ row_ptr, const int* __restrict__ col, int r, int c) {
  int lo = row_ptr[r], hi = row_ptr[r + 1] - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (col[mid] < c) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__global__ void k_emap(const int4* __restrict__ tets, int T, const int* __restrict__ row_ptr,
                       const int* __restrict__ col, int* emap) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)T * 10) return;
  const int e = (int)(i / 10), k = (int)(i % 10);
  const int4 t = tets[e];
  const int va = vtx(t, c_pa[k]), vb = vtx(t, c_pb[k]);
  emap[i] = find_slot(row_ptr, col, min(va, vb), max(va, vb));
}

__global__ void k_slot_count(const int* __restrict__ map, long long n, int* cnt) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) atomicAdd(&cnt[map[i]], 1);
}

__global__ void k_slot_fill(const int* __restrict__ map, long long n, const int* __restrict__ ptr, int* cursor,
                            int* list) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int s = map[i];
  list[ptr[s] + atomicAdd(&cursor[s], 1)] = (int)i;
}

__global__ void k_inverse_positions(const int* __restrict__ list, long long n, int* pos) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) pos[list[j]] = (int)j;
}

// m_v = sum over tets containing v of rho V / 4: the diagonal slot of v lists
// exactly the (tet, local diagonal pair) entries of its incident tets.
__global__ void k_mass(const int* __restrict__ ecptr, const int* __restrict__ elist,
                       const int* __restrict__ erow_ptr, const float* __restrict__ vol,
                       const double* __restrict__ rho, int N, double* mass) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N) return;
  const int d = erow_ptr[v];
  double m = 0.0;
  for (int j = ecptr[d]; j < ecptr[d + 1]; ++j) {
    const int e = elist[j] / 10;
    m += rho[e] * (double)vol[e] * 0.25;
  }
  mass[v] = m;
}

}  // namespace

void launch_check_tets(const int4* tets, int T, int N, int* flags, hipStream_t s) {
  if (T > 0) hipLaunchKernelGGL(k_check_tets, dim3(div_up(T, kBlock)), dim3(kBlock), 0, s, tets, T, N, flags);
}

void launch_rest_geometry(const int4* tets, const double* rest, const double* E, const double* nu,
                          const double* rho, int T, double* Dminv9, float* vol, float* mu, float* lam, int* flags,
                          hipStream_t s) {
  if (T > 0)
    hipLaunchKernelGGL(k_rest_geometry, dim3(div_up(T, kBlock)), dim3(kBlock), 0, s, tets, rest, E, nu, rho, T,
                       Dminv9, vol, mu, lam, flags);
}

void launch_elastic_pair_count(const int4* tets, int T, int* cnt, hipStream_t s) {
  if (T > 0) hipLaunchKernelGGL(k_pair_count, dim3(div_up(T, kBlock)), dim3(kBlock), 0, s, tets, T, cnt);
}

void launch_elastic_pair_fill(const int4* tets, int T, const int* ptr, int* cursor, int* keys, hipStream_t s) {
  if (T > 0)
    hipLaunchKernelGGL(k_pair_fill, dim3(div_up(T, kBlock)), dim3(kBlock), 0, s, tets, T, ptr, cursor, keys);
}

void launch_row_unique(int* keys, const int* kptr, int N, int* ucount, hipStream_t s) {
  hipLaunchKernelGGL(k_row_unique, dim3(div_up(N, kBlock)), dim3(kBlock), 0, s, keys, kptr, N, ucount);
}

void launch_row_write(const int* keys, const int* kptr, int N, const int* row_ptr, int* col, hipStream_t s) {
  hipLaunchKernelGGL(k_row_write, dim3(div_up(N, kBlock)), dim3(kBlock), 0, s, keys, kptr, N, row_ptr, col);
}

void launch_emap(const int4* tets, int T, const int* row_ptr, const int* col, int* emap, hipStream_t s) {
  if (T > 0)
    hipLaunchKernelGGL(k_emap, dim3(div_up(10LL * T, kBlock)), dim3(kBlock), 0, s, tets, T, row_ptr, col, emap);
}

void launch_slot_count(const int* map, long long n, int* cnt, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_slot_count, dim3(div_up(n, kBlock)), dim3(kBlock), 0, s, map, n, cnt);
}

void launch_slot_fill(const int* map, long long n, const int* ptr, int* cursor, int* list, hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(k_slot_fill, dim3(div_up(n, kBlock)), dim3(kBlock), 0, s, map, n, ptr, cursor, list);
}

void launch_inverse_positions(const int* list, long long n, int* pos, hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(k_inverse_positions, dim3(div_up(n, kBlock)), dim3(kBlock), 0, s, list, n, pos);
}

void launch_mass(const int* ecptr, const int* elist, const int* erow_ptr, const float* vol, const double* rho,
                 int N, double* mass, hipStream_t s) {
  hipLaunchKernelGGL(k_mass, dim3(div_up(N, kBlock)), dim3(kBlock), 0, s, ecptr, elist, erow_ptr, vol, rho, N,
                     mass);
}

}  // namespace bfal
