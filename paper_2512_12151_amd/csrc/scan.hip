// Integer primitives used to build the BSR pattern and its assembly order:
// exclusive prefix sum, per-segment sort, fill.  Wave64 scans through LDS.
#include "common.h"

namespace bfal {

namespace {

constexpr int kScanItems = 4;                       // items per thread
constexpr int kScanTile = kBlock * kScanItems;      // items per workgroup

__device__ inline int wave_inclusive_scan(int v) {
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    int t = __shfl_up(v, off, kWave);
    if (lane >= off) v += t;
  }
  return v;
}

__global__ void __launch_bounds__(kBlock) k_scan_tile(const int* __restrict__ in, int* out, long long n,
                                                      int* __restrict__ tile_sums) {
  __shared__ int wave_tot[kBlock / kWave];
  const long long base = (long long)blockIdx.x * kScanTile + (long long)threadIdx.x * kScanItems;
  int v[kScanItems];
  int s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = (base + k < n) ? in[base + k] : 0;
    s += v[k];
  }
  int inc = wave_inclusive_scan(s);
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  if (lane == kWave - 1) wave_tot[wid] = inc;
  __syncthreads();
  int wave_off = 0, total = 0;
#pragma unroll
  for (int w = 0; w < kBlock / kWave; ++w) {
    if (w < wid) wave_off += wave_tot[w];
    total += wave_tot[w];
  }
  int run = wave_off + inc - s;   // exclusive prefix of this thread
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

__global__ void k_add_tile_offsets(int* out, long long n, const int* __restrict__ tile_off) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += tile_off[i / kScanTile];
}

// Sorts every segment [ptr[i], ptr[i+1]) of keys ascending, one wavefront
// per segment: the segment is staged in LDS and each key is written to the
// position given by its rank (the smaller keys, and the equal ones before
// it), so no element waits for another.  A segment longer than kSortCap keys (rare: a
// vertex in very many constraints) is insertion-sorted by one lane.
constexpr int kSortWaves = 4;
constexpr int kSortCap = 256;

__global__ void __launch_bounds__(kSortWaves * 64) k_sort_segments(int* keys, const int* __restrict__ ptr, int nseg) {
  __shared__ int buf[kSortWaves][kSortCap];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int sg = blockIdx.x * kSortWaves + wave;
  const int b = sg < nseg ? ptr[sg] : 0;
  const int n = sg < nseg ? ptr[sg + 1] - b : 0;
  const bool staged = n > 1 && n <= kSortCap;
  if (staged)
    for (int i = lane; i < n; i += 64) buf[wave][i] = keys[b + i];
  __syncthreads();
  if (staged) {
    for (int i = lane; i < n; i += 64) {
      const int key = buf[wave][i];
      int rank = 0;
      for (int j = 0; j < n; ++j) {
        const int kj = buf[wave][j];
        rank += (kj < key || (kj == key && j < i)) ? 1 : 0;   // equal keys keep their order
      }
      keys[b + rank] = key;
    }
  } else if (n > kSortCap && lane == 0) {
    for (int j = b + 1; j < b + n; ++j) {
      const int key = keys[j];
      int k = j - 1;
      while (k >= b && keys[k] > key) { keys[k + 1] = keys[k]; --k; }
      keys[k + 1] = key;
    }
  }
}

__global__ void k_fill(int* a, int v, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

}  // namespace

size_t scan_tmp_ints(long long n) {
  size_t t = 0;
  while (n > 1) {
    long long nb = (n + kScanTile - 1) / kScanTile;
    t += (size_t)nb + 64;
    n = nb;
  }
  return t + 64;
}

void scan_exclusive(const int* in, int* out, long long n, int* total, int* tmp, hipStream_t s) {
  if (n <= 0) {
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(1), 0, s, total, 0, 1LL);
    return;
  }
  const long long nb = (n + kScanTile - 1) / kScanTile;
  if (nb == 1) {
    hipLaunchKernelGGL(k_scan_tile, dim3(1), dim3(kBlock), 0, s, in, out, n, total);
    return;
  }
  int* sums = tmp;
  hipLaunchKernelGGL(k_scan_tile, dim3((unsigned)nb), dim3(kBlock), 0, s, in, out, n, sums);
  scan_exclusive(sums, sums, nb, total, tmp + nb + 64, s);
  hipLaunchKernelGGL(k_add_tile_offsets, dim3((unsigned)div_up(n, kBlock)), dim3(kBlock), 0, s, out, n,
                     (const int*)sums);
}

void sort_segments(int* keys, const int* ptr, int nseg, hipStream_t s) {
  if (nseg <= 0) return;
  hipLaunchKernelGGL(k_sort_segments, dim3(div_up(nseg, kSortWaves)), dim3(kSortWaves * 64), 0, s, keys, ptr, nseg);
}

void fill_int(int* a, int v, long long n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)div_up(n, kBlock)), dim3(kBlock), 0, s, a, v, n);
}

}  // namespace bfal
