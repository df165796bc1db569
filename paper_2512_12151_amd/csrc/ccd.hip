// Collision side of the time step (Algorithm 1's MaxStepSize and Algorithm 3,
// UpdateActiveSet): which surface primitive pairs collide along the straight
// path x -> x_hat, and when.
//
// Broad phase: a linear BVH (Karras 2012) over the swept boxes of the
// surface triangles (point-triangle queries, one thread per surface vertex)
// and of the surface edges (edge-edge queries, one thread per edge, pairs
// (i, j) with i < j).  Boxes are FP32, rounded outward from the FP64
// positions, so the tree test is conservative; every pair it reports is
// tested again exactly in FP64 (swept boxes within delta on every axis) and
// pairs sharing a vertex are skipped.
//
// Narrow phase: additive CCD (Li, Kaufman and Jiang 2021) in FP64, run by the
// querying thread as soon as a pair passes the exact test, so candidates are
// never stored: remove the pair's common translation, bound the rate at which
// the distance can shrink by l_p (largest displacement of a vertex of each
// primitive, summed), and advance by steps that cannot close the gap --
// (1 - s) d0 / l_p first, then 0.9 d / l_p -- until a step lands below s d0
// (collision at the time before that step) or passes t = 1.  After 10^4 steps
// a pair counts as colliding at the time reached; a pair at distance 0 at
// t = 0 collides at 0.  Colliding pairs are appended with their time.
//
// The active-set update then keeps, of the colliding pairs not already
// constrained, those whose time is the earliest of one of their vertices
// (per-vertex atomicMin over the FP64 bit patterns, which order like the
// values for t >= 0; "earliest" up to 1e-9 relative, the times' rounding),
// sorts them into a canonical order, and rebuilds the
// constraint arrays: surviving current PT constraints (gamma >= 0.01, in
// their order), new PT pairs, surviving current EE constraints, new EE pairs.
#include <hipcub/hipcub.hpp>

#include "common.h"

namespace bfal {

namespace {

constexpr int kCcdBlock = 256;
constexpr int kAccdMaxSteps = 10000;
constexpr int kStackDepth = 64;

struct d3 {
  double x, y, z;
};
__device__ inline d3 ld3(const double* p, int v) { return {p[3LL * v], p[3LL * v + 1], p[3LL * v + 2]}; }
__device__ inline d3 sub(d3 a, d3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline d3 add(d3 a, d3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ inline d3 mul(d3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
__device__ inline double dot(d3 a, d3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline double norm(d3 a) { return sqrt(dot(a, a)); }
__device__ inline double clamp01(double t) { return t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t); }
__device__ inline double seg_param(d3 p, d3 u, d3 v) {
  const d3 e = sub(v, u);
  return clamp01(dot(sub(p, u), e) / dot(e, e));
}

// Distance from p to the closed triangle (t0, t1, t2): the interior
// projection when it lies inside, else the nearest of the three edge points.
__device__ inline double pt_dist(d3 p, d3 t0, d3 t1, d3 t2) {
  const d3 e1 = sub(t1, t0), e2 = sub(t2, t0), r = sub(p, t0);
  const double a11 = dot(e1, e1), a12 = dot(e1, e2), a22 = dot(e2, e2);
  const double r1 = dot(e1, r), r2 = dot(e2, r);
  const double det = a11 * a22 - a12 * a12;
  const double u = (a22 * r1 - a12 * r2) / det, v = (a11 * r2 - a12 * r1) / det;
  double best = INFINITY;
  if (u >= 0.0 && v >= 0.0 && u + v <= 1.0) best = norm(sub(p, add(t0, add(mul(e1, u), mul(e2, v)))));
  const d3 T[3] = {t0, t1, t2};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const d3 a = T[k], b = T[(k + 1) % 3];
    const double s = seg_param(p, a, b);
    best = fmin(best, norm(sub(p, add(a, mul(sub(b, a), s)))));
  }
  return best;
}

// Distance between segments a0 a1 and b0 b1: the interior stationary point
// when it lies in the unit square, else the best of the four clamped ones.
__device__ inline double ee_dist(d3 a0, d3 a1, d3 b0, d3 b1) {
  const d3 ea = sub(a1, a0), eb = sub(b1, b0), r = sub(a0, b0);
  const double aa = dot(ea, ea), bb = dot(eb, eb), ab = dot(ea, eb);
  const double ar = dot(ea, r), br = dot(eb, r);
  const double det = aa * bb - ab * ab;
  double best = INFINITY;
  if (det > 0.0) {
    const double s = (-ar * bb + ab * br) / det, t = (aa * br - ab * ar) / det;
    if (s >= 0.0 && s <= 1.0 && t >= 0.0 && t <= 1.0) best = norm(sub(add(a0, mul(ea, s)), add(b0, mul(eb, t))));
  }
  const double cs[4] = {0.0, 1.0, seg_param(b0, a0, a1), seg_param(b1, a0, a1)};
  const double ct[4] = {seg_param(a0, b0, b1), seg_param(a1, b0, b1), 0.0, 1.0};
#pragma unroll
  for (int k = 0; k < 4; ++k) best = fmin(best, norm(sub(add(a0, mul(ea, cs[k])), add(b0, mul(eb, ct[k])))));
  return best;
}

template <bool kEE>
__device__ inline double pair_dist(const d3 X[4]) {
  return kEE ? ee_dist(X[0], X[1], X[2], X[3]) : pt_dist(X[0], X[1], X[2], X[3]);
}

// Additive CCD of one pair along X0 -> X1; returns the collision time, or a
// negative value when the pair does not collide in [0, 1].
template <bool kEE>
__device__ double accd(const d3 X0[4], const d3 X1[4], double s) {
  d3 P[4], X[4];
  d3 m = {0.0, 0.0, 0.0};
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    P[a] = sub(X1[a], X0[a]);
    m = add(m, P[a]);
  }
  m = mul(m, 0.25);
  double la = 0.0, lb = 0.0;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    P[a] = sub(P[a], m);
    X[a] = X0[a];
    const double n = norm(P[a]);
    if (a < (kEE ? 2 : 1)) la = fmax(la, n);
    else lb = fmax(lb, n);
  }
  const double lp = la + lb;
  const double d0 = pair_dist<kEE>(X);
  if (d0 == 0.0) return 0.0;
  if (!(lp > 0.0)) return -1.0;
  const double gap = s * d0;
  double t = 0.0, tl = (1.0 - s) * d0 / lp;
  for (int it = 0; it < kAccdMaxSteps; ++it) {
#pragma unroll
    for (int a = 0; a < 4; ++a) X[a] = add(X[a], mul(P[a], tl));
    const double d = pair_dist<kEE>(X);
    if (it > 0 && d < gap) return t;
    t += tl;
    if (t > 1.0) return -1.0;
    tl = 0.9 * d / lp;
  }
  return t;   // step cap: collision at the time reached
}

// ---------------------------------------------------------------- boxes

struct Box {
  float lo[3], hi[3];
};

__device__ inline void box_of(const double* x, const double* xh, const int* v, int k, double lo[3], double hi[3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    lo[c] = INFINITY;
    hi[c] = -INFINITY;
  }
  for (int a = 0; a < k; ++a) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double p = x[3LL * v[a] + c], q = xh[3LL * v[a] + c];
      lo[c] = fmin(lo[c], fmin(p, q));
      hi[c] = fmax(hi[c], fmax(p, q));
    }
  }
}

// FP32 swept boxes of the primitives (k vertices each, ids AoS [n][k] in
// stride st), rounded outward; and their centres for the Morton codes.
__global__ void k_prim_boxes(int n, const int* __restrict__ ids, int k, int st, const double* __restrict__ x,
                             const double* __restrict__ xh, Box* __restrict__ box) {
  const int i = blockIdx.x * kCcdBlock + threadIdx.x;
  if (i >= n) return;
  int v[3];
  for (int a = 0; a < k; ++a) v[a] = ids[(long long)st * i + a];
  double lo[3], hi[3];
  box_of(x, xh, v, k, lo, hi);
  Box b;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    b.lo[c] = __double2float_rd(lo[c]);
    b.hi[c] = __double2float_ru(hi[c]);
  }
  box[i] = b;
}

// Bounds of all leaf boxes: per-workgroup partial boxes, then one workgroup
// combines them.
__global__ void k_bounds_part(int n, const Box* __restrict__ box, Box* __restrict__ part) {
  __shared__ float red[6][kCcdBlock];
  float b[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
  for (int i = blockIdx.x * kCcdBlock + threadIdx.x; i < n; i += gridDim.x * kCcdBlock) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      b[c] = fminf(b[c], box[i].lo[c]);
      b[3 + c] = fmaxf(b[3 + c], box[i].hi[c]);
    }
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) red[c][threadIdx.x] = b[c];
  __syncthreads();
  for (int off = kCcdBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off)
#pragma unroll
      for (int c = 0; c < 6; ++c)
        red[c][threadIdx.x] = c < 3 ? fminf(red[c][threadIdx.x], red[c][threadIdx.x + off])
                                    : fmaxf(red[c][threadIdx.x], red[c][threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    Box o;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      o.lo[c] = red[c][0];
      o.hi[c] = red[3 + c][0];
    }
    part[blockIdx.x] = o;
  }
}

__device__ inline unsigned int spread10(unsigned int v) {
  v &= 1023u;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

// 64-bit sort keys: the 30-bit Morton code of the box centre (in the scene
// bounds) above the primitive index, so equal codes order by index.
__global__ void k_morton(int n, const Box* __restrict__ box, const Box* __restrict__ part, int nparts,
                         unsigned long long* __restrict__ key) {
  const int i = blockIdx.x * kCcdBlock + threadIdx.x;
  if (i >= n) return;
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int p = 0; p < nparts; ++p)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      lo[c] = fminf(lo[c], part[p].lo[c]);
      hi[c] = fmaxf(hi[c], part[p].hi[c]);
    }
  unsigned int code = 0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float ext = hi[c] - lo[c];
    const float u = ext > 0.f ? (0.5f * (box[i].lo[c] + box[i].hi[c]) - lo[c]) / ext : 0.f;
    const unsigned int q = (unsigned int)fminf(fmaxf(u * 1024.f, 0.f), 1023.f);
    code |= spread10(q) << (2 - c);
  }
  key[i] = ((unsigned long long)code << 32) | (unsigned int)i;
}

// ------------------------------------------------------------ tree build

__device__ inline int common_prefix(const unsigned long long* key, int n, int i, int j) {
  if (j < 0 || j >= n) return -1;
  return __clzll(key[i] ^ key[j]);   // keys are unique (index in the low bits)
}

// Karras' construction: internal node i (0 <= i < n - 1) covers the key range
// found by a binary search on the common-prefix length; children are internal
// nodes or leaves (leaf k is node n - 1 + k).
__global__ void k_karras(int n, const unsigned long long* __restrict__ key, int2* __restrict__ child,
                         int2* __restrict__ range) {
  const int i = blockIdx.x * kCcdBlock + threadIdx.x;
  if (i >= n - 1) return;
  const int d = common_prefix(key, n, i, i + 1) - common_prefix(key, n, i, i - 1) >= 0 ? 1 : -1;
  const int dmin = common_prefix(key, n, i, i - d);
  int lmax = 2;
  while (common_prefix(key, n, i, i + lmax * d) > dmin) lmax *= 2;
  int l = 0;
  for (int t = lmax / 2; t >= 1; t /= 2)
    if (common_prefix(key, n, i, i + (l + t) * d) > dmin) l += t;
  const int j = i + l * d;
  const int dnode = common_prefix(key, n, i, j);
  int s = 0;
  for (int t = (l + 1) / 2;; t = (t + 1) / 2) {
    if (common_prefix(key, n, i, i + (s + t) * d) > dnode) s += t;
    if (t == 1) break;
  }
  const int g = i + s * d + (d < 0 ? -1 : 0);
  const int left = (min(i, j) == g) ? (n - 1 + g) : g;
  const int right = (max(i, j) == g + 1) ? (n - 1 + g + 1) : g + 1;
  child[i] = make_int2(left, right);
  range[i] = make_int2(min(i, j), max(i, j));
}

// Node boxes without atomics: an internal node covers the contiguous range
// [a, b] of sorted leaves, so its box is the union of two overlapping runs of
// 2^m leaves (2^m <= b - a + 1 < 2^(m+1)), read from a sparse table whose
// level k holds the union of the 2^k leaves starting at each position.
__device__ inline Box box_union(const Box& a, const Box& b) {
  Box u;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    u.lo[q] = fminf(a.lo[q], b.lo[q]);
    u.hi[q] = fmaxf(a.hi[q], b.hi[q]);
  }
  return u;
}

// Level 0 of the table and the leaf nodes: the primitive boxes in key order.
__global__ void k_leaf_boxes(int n, const unsigned long long* __restrict__ key, const Box* __restrict__ pbox,
                             Box* __restrict__ level0, Box* __restrict__ node) {
  const int k = blockIdx.x * kCcdBlock + threadIdx.x;
  if (k >= n) return;
  const Box b = pbox[(int)(key[k] & 0xffffffffu)];
  level0[k] = b;
  node[n - 1 + k] = b;
}

// Level k from level k - 1 (run length h = 2^(k-1)): entries i + 2h <= n.
__global__ void k_sparse_level(int n, int h, const Box* __restrict__ prev, Box* __restrict__ next) {
  const int i = blockIdx.x * kCcdBlock + threadIdx.x;
  if (i + 2 * h > n) return;
  next[i] = box_union(prev[i], prev[i + h]);
}

__global__ void k_node_boxes(int n, const int2* __restrict__ range, const Box* __restrict__ table,
                             Box* __restrict__ node) {
  const int i = blockIdx.x * kCcdBlock + threadIdx.x;
  if (i >= n - 1) return;
  const int2 r = range[i];
  const int len = r.y - r.x + 1;
  const int m = 31 - __clz(len);
  const Box* lv = table + (long long)m * n;
  node[i] = box_union(lv[r.x], lv[r.y - (1 << m) + 1]);
}

// ------------------------------------------------------------ queries

__device__ inline bool overlap(const Box& a, const float lo[3], const float hi[3]) {
  return a.lo[0] <= hi[0] && lo[0] <= a.hi[0] && a.lo[1] <= hi[1] && lo[1] <= a.hi[1] && a.lo[2] <= hi[2] &&
         lo[2] <= a.hi[2];
}

// The oracle's exact test: FP64 swept boxes within delta on every axis.
__device__ inline bool near_exact(const double alo[3], const double ahi[3], const double blo[3], const double bhi[3],
                                  double delta) {
  bool ok = true;
#pragma unroll
  for (int c = 0; c < 3; ++c) ok = ok && (alo[c] - delta <= bhi[c]) && (blo[c] - delta <= ahi[c]);
  return ok;
}

struct QueryOut {
  int* count;              // [0] colliding pairs, [1] traversal-stack overflow flag, [2..3] candidate count (u64)
  int cap;
  int2* pairs;             // (query primitive, tree primitive)
  double* toc;
};

// One thread per query primitive (a surface vertex for PT, an edge for EE):
// traverse the tree of the other kind, test the exact condition, run ACCD.
template <bool kEE>
__global__ void __launch_bounds__(kCcdBlock)
k_query(int nq, const int* __restrict__ qids, int nt, const int* __restrict__ tids, const int2* __restrict__ child,
        const Box* __restrict__ node, const unsigned long long* __restrict__ key, const double* __restrict__ x,
        const double* __restrict__ xh, double delta, double s, QueryOut out) {
  const int i = blockIdx.x * kCcdBlock + threadIdx.x;
  long long cand = 0;
  if (i < nq && nt > 0) {
    constexpr int kq = kEE ? 2 : 1;
    constexpr int kt = kEE ? 2 : 3;
    int qv[kq];
#pragma unroll
    for (int a = 0; a < kq; ++a) qv[a] = qids[(long long)kq * i + a];
    double qlo[3], qhi[3];
    box_of(x, xh, qv, kq, qlo, qhi);
    float flo[3], fhi[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      flo[c] = __double2float_rd(qlo[c] - delta);
      fhi[c] = __double2float_ru(qhi[c] + delta);
    }
    int stack[kStackDepth];
    int sp = 0;
    stack[sp++] = 0;   // root (a leaf when nt == 1)
    while (sp > 0) {
      const int v = stack[--sp];
      if (!overlap(node[v], flo, fhi)) continue;
      if (v < nt - 1) {
        const int2 c = child[v];
        if (sp + 2 > kStackDepth) {   // cannot happen for trees of depth < 63; reported, never dropped silently
          out.count[1] = 1;
          break;
        }
        stack[sp++] = c.y;
        stack[sp++] = c.x;
        continue;
      }
      const int j = (int)(key[v - (nt - 1)] & 0xffffffffu);   // tree primitive index
      if (kEE && j <= i) continue;
      int tv[kt];
#pragma unroll
      for (int a = 0; a < kt; ++a) tv[a] = tids[(long long)kt * j + a];
      bool share = false;
#pragma unroll
      for (int a = 0; a < kq; ++a)
#pragma unroll
        for (int b = 0; b < kt; ++b) share = share || qv[a] == tv[b];
      if (share) continue;
      double tlo[3], thi[3];
      box_of(x, xh, tv, kt, tlo, thi);
      if (!near_exact(qlo, qhi, tlo, thi, delta)) continue;
      ++cand;
      int ids[4];
      if (kEE) {
        ids[0] = qv[0]; ids[1] = qv[1]; ids[2] = tv[0]; ids[3] = tv[1];
      } else {
        ids[0] = qv[0]; ids[1] = tv[0]; ids[2] = tv[1]; ids[3] = tv[2];
      }
      d3 X0[4], X1[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        X0[a] = ld3(x, ids[a]);
        X1[a] = ld3(xh, ids[a]);
      }
      const double t = accd<kEE>(X0, X1, s);
      if (t >= 0.0) {
        const int slot = atomicAdd(out.count, 1);
        if (slot < out.cap) {
          out.pairs[slot] = make_int2(i, j);
          out.toc[slot] = t;
        }
      }
    }
  }
  // candidate count of the workgroup (statistics)
  __shared__ long long red[kCcdBlock / kWave];
  long long c = cand;
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) c += __shfl_xor(c, off, kWave);
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long tot = 0;
    for (int w = 0; w < kCcdBlock / kWave; ++w) tot += red[w];
    if (tot) atomicAdd(reinterpret_cast<unsigned long long*>(out.count + 2), (unsigned long long)tot);
  }
}

// Canonical 64-bit order of a colliding pair: query index above tree index
// (PT: surface-vertex position, which follows the vertex id, then triangle;
// EE: edge i < edge j).
__global__ void k_pair_keys(int n, const int2* __restrict__ pairs, unsigned long long* __restrict__ key,
                            int* __restrict__ idx) {
  const int i = blockIdx.x * kCcdBlock + threadIdx.x;
  if (i >= n) return;
  key[i] = ((unsigned long long)(unsigned int)pairs[i].x << 32) | (unsigned int)pairs[i].y;
  idx[i] = i;
}

// ------------------------------------------------------------ active set

__device__ inline void sort3(int& a, int& b, int& c) {
  if (a > b) { const int t = a; a = b; b = t; }
  if (b > c) { const int t = b; b = c; c = t; }
  if (a > b) { const int t = a; a = b; b = t; }
}

// Canonical 4-int key of a constraint: PT (p, sorted triangle); EE (sorted
// edges, the smaller edge first).
__device__ inline int4 canon(int4 t, bool ee) {
  if (!ee) {
    sort3(t.y, t.z, t.w);
    return t;
  }
  int a0 = min(t.x, t.y), a1 = max(t.x, t.y), b0 = min(t.z, t.w), b1 = max(t.z, t.w);
  if (a0 > b0 || (a0 == b0 && a1 > b1)) {
    const int u0 = a0, u1 = a1;
    a0 = b0; a1 = b1; b0 = u0; b1 = u1;
  }
  return make_int4(a0, a1, b0, b1);
}

__device__ inline unsigned long long hash4(int4 k, bool ee) {
  unsigned long long h = ee ? 0x9E3779B97F4A7C15ull : 0xC2B2AE3D27D4EB4Full;
  const int v[4] = {k.x, k.y, k.z, k.w};
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    h ^= (unsigned long long)(unsigned int)v[a] + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
    h *= 0xFF51AFD7ED558CCDull;
  }
  return h ^ (h >> 33);
}

// Open-addressing set of the current constraints (slot value = constraint index).
__global__ void k_hash_insert(int n_c, int n_pt, const int4* __restrict__ ids, int* __restrict__ table,
                              unsigned int mask) {
  const int i = blockIdx.x * kCcdBlock + threadIdx.x;
  if (i >= n_c) return;
  const bool ee = i >= n_pt;
  unsigned int h = (unsigned int)hash4(canon(ids[i], ee), ee) & mask;
  while (atomicCAS(&table[h], -1, i) != -1) h = (h + 1) & mask;
}

__device__ inline bool hash_find(int4 key, bool ee, int n_pt, const int4* __restrict__ ids,
                                 const int* __restrict__ table, unsigned int mask) {
  unsigned int h = (unsigned int)hash4(key, ee) & mask;
  while (true) {
    const int c = table[h];
    if (c < 0) return false;
    if ((c >= n_pt) == ee) {
      const int4 k = canon(ids[c], ee);
      if (k.x == key.x && k.y == key.y && k.z == key.z && k.w == key.w) return true;
    }
    h = (h + 1) & mask;
  }
}

__device__ inline int4 pair_ids(bool ee, int2 pr, const int* __restrict__ qids, const int* __restrict__ tids) {
  if (ee) return make_int4(qids[2LL * pr.x], qids[2LL * pr.x + 1], tids[2LL * pr.y], tids[2LL * pr.y + 1]);
  return make_int4(qids[pr.x], tids[3LL * pr.y], tids[3LL * pr.y + 1], tids[3LL * pr.y + 2]);
}

// New colliding pairs (sorted order): not in the current set; their times
// lower the per-vertex earliest time.
// An edge pair (near-)parallel at x: its distance gradient is not unique and
// the linearization rejects it, so it cannot enter the active set.
__device__ inline bool ee_parallel(const double* __restrict__ x, int4 id) {
  const d3 ea = sub(ld3(x, id.y), ld3(x, id.x)), eb = sub(ld3(x, id.w), ld3(x, id.z));
  const d3 cr = {ea.y * eb.z - ea.z * eb.y, ea.z * eb.x - ea.x * eb.z, ea.x * eb.y - ea.y * eb.x};
  return dot(cr, cr) < 1e-8 * dot(ea, ea) * dot(eb, eb);
}

__global__ void k_new_and_tv(int n, bool ee, const int* __restrict__ order, const int2* __restrict__ pairs,
                             const double* __restrict__ toc, const int* __restrict__ qids,
                             const int* __restrict__ tids, int n_pt, const int4* __restrict__ cids,
                             const int* __restrict__ table, unsigned int mask, const double* __restrict__ x,
                             int* __restrict__ is_new, unsigned long long* __restrict__ tv) {
  const int i = blockIdx.x * kCcdBlock + threadIdx.x;
  if (i >= n) return;
  const int o = order[i];
  const int4 id = pair_ids(ee, pairs[o], qids, tids);
  const bool found = (ee && ee_parallel(x, id)) ||
                     (table != nullptr && hash_find(canon(id, ee), ee, n_pt, cids, table, mask));
  is_new[i] = found ? 0 : 1;
  if (!found) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(toc[o]);
    atomicMin(&tv[id.x], b);
    atomicMin(&tv[id.y], b);
    atomicMin(&tv[id.z], b);
    atomicMin(&tv[id.w], b);
  }
}

__global__ void k_keep_new(int n, bool ee, const int* __restrict__ order, const int2* __restrict__ pairs,
                           const double* __restrict__ toc, const int* __restrict__ qids, const int* __restrict__ tids,
                           const unsigned long long* __restrict__ tv, int* __restrict__ keep) {
  const int i = blockIdx.x * kCcdBlock + threadIdx.x;
  if (i >= n) return;
  if (!keep[i]) return;   // holds is_new on entry
  const int o = order[i];
  const int4 id = pair_ids(ee, pairs[o], qids, tids);
  // the earliest time of a vertex, up to the times' own rounding
  const double t = toc[o];
  auto earliest = [&](int v) { return t <= __longlong_as_double((long long)tv[v]) * (1.0 + 1e-9); };
  keep[i] = (earliest(id.x) || earliest(id.y) || earliest(id.z) || earliest(id.w)) ? 1 : 0;
}

__global__ void k_keep_current(int lo, int hi, const double* __restrict__ gam, double gmin, int* __restrict__ keep) {
  const int i = blockIdx.x * kCcdBlock + threadIdx.x;
  if (lo + i < hi) keep[i] = gam[lo + i] >= gmin ? 1 : 0;
}

// Scatter the surviving current constraints of [lo, hi) to out + pos.
__global__ void k_scatter_current(int lo, int hi, const int* __restrict__ keep, const int* __restrict__ pos,
                                  int base, const int4* __restrict__ ids, const double* __restrict__ lam,
                                  const double* __restrict__ gam, int4* __restrict__ oids, double* __restrict__ olam,
                                  double* __restrict__ ogam) {
  const int i = blockIdx.x * kCcdBlock + threadIdx.x;
  if (lo + i >= hi || !keep[i]) return;
  const int o = base + pos[i];
  oids[o] = ids[lo + i];
  olam[o] = lam[lo + i];
  ogam[o] = gam[lo + i];
}

__global__ void k_scatter_new(int n, bool ee, const int* __restrict__ keep, const int* __restrict__ pos, int base,
                              const int* __restrict__ order, const int2* __restrict__ pairs,
                              const int* __restrict__ qids, const int* __restrict__ tids, int4* __restrict__ oids,
                              double* __restrict__ olam, double* __restrict__ ogam) {
  const int i = blockIdx.x * kCcdBlock + threadIdx.x;
  if (i >= n || !keep[i]) return;
  const int o = base + pos[i];
  oids[o] = pair_ids(ee, pairs[order[i]], qids, tids);
  olam[o] = 0.0;
  ogam[o] = 1.0;
}

__global__ void k_pair_rows(int n, bool ee, const int2* __restrict__ pairs, const int* __restrict__ qids,
                            const int* __restrict__ tids, int4* __restrict__ rows) {
  const int i = blockIdx.x * kCcdBlock + threadIdx.x;
  if (i < n) rows[i] = pair_ids(ee, pairs[i], qids, tids);
}

__global__ void k_fill_u64(unsigned long long* a, unsigned long long v, int n) {
  const int i = blockIdx.x * kCcdBlock + threadIdx.x;
  if (i < n) a[i] = v;
}

// ------------------------------------------------------------ step size

// Per workgroup the smallest collision time of a pair list.
__global__ void k_min_toc(int n, const double* __restrict__ toc, double* __restrict__ part) {
  __shared__ double red[kCcdBlock];
  double m = 1.0;
  for (int i = blockIdx.x * kCcdBlock + threadIdx.x; i < n; i += gridDim.x * kCcdBlock) m = fmin(m, toc[i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int off = kCcdBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__device__ inline double det3(d3 a, d3 b, d3 c) {   // det of the matrix with columns a, b, c
  return a.x * (b.y * c.z - b.z * c.y) - b.x * (a.y * c.z - a.z * c.y) + c.x * (a.y * b.z - a.z * b.y);
}

// Per tet the first t in (0, 1] where det D_s(t) / det D_s(0) falls to s (1 if
// none), for either orientation of the tet: the cubic's coefficients by
// interpolation at t = 0, 1/3, 2/3, 1, taken times the sign of det D_s(0); its
// derivative's roots split [0, 1] into monotone pieces, the first piece whose
// end falls to the level s |det D_s(0)| is bisected (60 halvings, the lower end
// kept).
__global__ void k_inversion_bound(int T, const int4* __restrict__ tets, const double* __restrict__ x,
                                  const double* __restrict__ xh, double s, double* __restrict__ part) {
  __shared__ double red[kCcdBlock];
  const int e = blockIdx.x * kCcdBlock + threadIdx.x;
  double out = 1.0;
  if (e < T) {
    const int4 t = tets[e];
    const d3 p0 = ld3(x, t.x), p1 = ld3(x, t.y), p2 = ld3(x, t.z), p3 = ld3(x, t.w);
    const d3 q0 = ld3(xh, t.x), q1 = ld3(xh, t.y), q2 = ld3(xh, t.z), q3 = ld3(xh, t.w);
    const d3 a0 = sub(p1, p0), b0 = sub(p2, p0), c0 = sub(p3, p0);
    const d3 da = sub(sub(q1, q0), a0), db = sub(sub(q2, q0), b0), dc = sub(sub(q3, q0), c0);
    auto J = [&](double tt) { return det3(add(a0, mul(da, tt)), add(b0, mul(db, tt)), add(c0, mul(dc, tt))); };
    const double f0 = J(0.0), f1 = J(1.0 / 3.0), f2 = J(2.0 / 3.0), f3 = J(1.0);
    // Newton form at 0, 1/3, 2/3, 1 (h = 1/3), expanded to the monomial coefficients
    const double h = 1.0 / 3.0;
    const double d1a = (f1 - f0) / h, d1b = (f2 - f1) / h, d1c = (f3 - f2) / h;
    const double d2a = (d1b - d1a) / (2 * h), d2b = (d1c - d1b) / (2 * h);
    const double d3v = (d2b - d2a) / (3 * h);
    // p(t) = f0 + d1a t + d2a t (t - h) + d3v t (t - h)(t - 2h)
    const double sg = f0 < 0.0 ? -1.0 : 1.0;
    const double c3 = sg * d3v;
    const double c2 = sg * (d2a - 3 * h * d3v);
    const double c1 = sg * (d1a - h * d2a + 2 * h * h * d3v);
    const double c0v = sg * f0;
    const double level = s * c0v;
    auto F = [&](double tt) { return ((c3 * tt + c2) * tt + c1) * tt + c0v - level; };
    double knots[4];
    int nk = 0;
    knots[nk++] = 0.0;
    const double A = 3 * c3, B = 2 * c2, C = c1;
    double r[2];
    int nr = 0;
    if (A != 0.0) {
      const double disc = B * B - 4 * A * C;
      if (disc >= 0.0) {
        const double sq = sqrt(disc);
        r[0] = (-B - sq) / (2 * A);
        r[1] = (-B + sq) / (2 * A);
        if (r[0] > r[1]) { const double u = r[0]; r[0] = r[1]; r[1] = u; }
        nr = 2;
      }
    } else if (B != 0.0) {
      r[0] = -C / B;
      nr = 1;
    }
    for (int k = 0; k < nr; ++k)
      if (r[k] > 0.0 && r[k] < 1.0) knots[nk++] = r[k];
    knots[nk++] = 1.0;
    for (int k = 0; k + 1 < nk; ++k) {
      double lo = knots[k], hi = knots[k + 1];
      if (F(hi) <= 0.0) {
        for (int it = 0; it < 60; ++it) {
          const double mid = 0.5 * (lo + hi);
          if (F(mid) > 0.0) lo = mid;
          else hi = mid;
        }
        out = lo;
        break;
      }
    }
  }
  red[threadIdx.x] = out;
  __syncthreads();
  for (int off = kCcdBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

}  // namespace

// ---------------------------------------------------------------- launchers

size_t ccd_sort_tmp_bytes(int n) {
  size_t bytes = 0;
  (void)hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (unsigned long long*)nullptr, (unsigned long long*)nullptr,
                                     (int*)nullptr, (int*)nullptr, n, 0, 64, (hipStream_t)0);
  return bytes;
}

hipError_t ccd_sort_pairs(void* tmp, size_t tmp_bytes, const unsigned long long* kin, unsigned long long* kout,
                          const int* vin, int* vout, int n, hipStream_t s) {
  return hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, kin, kout, vin, vout, n, 0, 64, s);
}

size_t ccd_sort_keys_tmp_bytes(int n) {
  size_t bytes = 0;
  (void)hipcub::DeviceRadixSort::SortKeys(nullptr, bytes, (unsigned long long*)nullptr, (unsigned long long*)nullptr, n, 0,
                                    64, (hipStream_t)0);
  return bytes;
}

hipError_t ccd_sort_keys(void* tmp, size_t tmp_bytes, const unsigned long long* kin, unsigned long long* kout, int n,
                         hipStream_t s) {
  return hipcub::DeviceRadixSort::SortKeys(tmp, tmp_bytes, kin, kout, n, 0, 64, s);
}

void launch_prim_boxes(int n, const int* ids, int k, const double* x, const double* xh, void* box, hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(k_prim_boxes, dim3(div_up(n, kCcdBlock)), dim3(kCcdBlock), 0, s, n, ids, k, k, x, xh,
                       static_cast<Box*>(box));
}

int ccd_bounds_parts(int n) { return std::min(div_up(n, kCcdBlock), 256); }

void launch_morton(int n, const void* box, void* part, unsigned long long* key, hipStream_t s) {
  if (n <= 0) return;
  const int np = ccd_bounds_parts(n);
  hipLaunchKernelGGL(k_bounds_part, dim3(np), dim3(kCcdBlock), 0, s, n, static_cast<const Box*>(box),
                     static_cast<Box*>(part));
  hipLaunchKernelGGL(k_morton, dim3(div_up(n, kCcdBlock)), dim3(kCcdBlock), 0, s, n, static_cast<const Box*>(box),
                     static_cast<const Box*>(part), np, key);
}

int ccd_table_levels(int n) {
  int L = 1;
  while ((2LL << (L - 1)) <= n) ++L;   // levels 0 .. L-1 with 2^(L-1) <= n
  return L;
}

void launch_build_tree(int n, const unsigned long long* key, const void* pbox, int2* child, int2* range, void* node,
                       void* table, hipStream_t s) {
  if (n <= 0) return;
  Box* T = static_cast<Box*>(table);
  hipLaunchKernelGGL(k_leaf_boxes, dim3(div_up(n, kCcdBlock)), dim3(kCcdBlock), 0, s, n, key,
                     static_cast<const Box*>(pbox), T, static_cast<Box*>(node));
  if (n == 1) return;
  hipLaunchKernelGGL(k_karras, dim3(div_up(n - 1, kCcdBlock)), dim3(kCcdBlock), 0, s, n, key, child, range);
  const int L = ccd_table_levels(n);
  for (int k = 1; k < L; ++k) {
    const int h = 1 << (k - 1);
    hipLaunchKernelGGL(k_sparse_level, dim3(div_up(n - 2 * h + 1, kCcdBlock)), dim3(kCcdBlock), 0, s, n, h,
                       T + (long long)(k - 1) * n, T + (long long)k * n);
  }
  hipLaunchKernelGGL(k_node_boxes, dim3(div_up(n - 1, kCcdBlock)), dim3(kCcdBlock), 0, s, n, range, T,
                     static_cast<Box*>(node));
}

void launch_query(bool ee, int nq, const int* qids, int nt, const int* tids, const int2* child, const void* node,
                  const unsigned long long* key, const double* x, const double* xh, double delta, double sep,
                  int* count, int cap, int2* pairs, double* toc, hipStream_t s) {
  if (nq <= 0) return;
  QueryOut out{count, cap, pairs, toc};
  if (ee)
    hipLaunchKernelGGL(k_query<true>, dim3(div_up(nq, kCcdBlock)), dim3(kCcdBlock), 0, s, nq, qids, nt, tids, child,
                       static_cast<const Box*>(node), key, x, xh, delta, sep, out);
  else
    hipLaunchKernelGGL(k_query<false>, dim3(div_up(nq, kCcdBlock)), dim3(kCcdBlock), 0, s, nq, qids, nt, tids, child,
                       static_cast<const Box*>(node), key, x, xh, delta, sep, out);
}

void launch_pair_keys(int n, const int2* pairs, unsigned long long* key, int* idx, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_pair_keys, dim3(div_up(n, kCcdBlock)), dim3(kCcdBlock), 0, s, n, pairs, key, idx);
}

void launch_hash_insert(int n_c, int n_pt, const int4* ids, int* table, unsigned int mask, hipStream_t s) {
  if (n_c > 0)
    hipLaunchKernelGGL(k_hash_insert, dim3(div_up(n_c, kCcdBlock)), dim3(kCcdBlock), 0, s, n_c, n_pt, ids, table,
                       mask);
}

void launch_pair_rows(int n, bool ee, const int2* pairs, const int* qids, const int* tids, int4* rows, hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(k_pair_rows, dim3(div_up(n, kCcdBlock)), dim3(kCcdBlock), 0, s, n, ee, pairs, qids, tids, rows);
}

void launch_fill_u64(unsigned long long* a, unsigned long long v, int n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_fill_u64, dim3(div_up(n, kCcdBlock)), dim3(kCcdBlock), 0, s, a, v, n);
}

void launch_new_and_tv(int n, bool ee, const int* order, const int2* pairs, const double* toc, const int* qids,
                       const int* tids, int n_pt, const int4* cids, const int* table, unsigned int mask,
                       const double* x, int* is_new, unsigned long long* tv, hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(k_new_and_tv, dim3(div_up(n, kCcdBlock)), dim3(kCcdBlock), 0, s, n, ee, order, pairs, toc,
                       qids, tids, n_pt, cids, table, mask, x, is_new, tv);
}

void launch_keep_new(int n, bool ee, const int* order, const int2* pairs, const double* toc, const int* qids,
                     const int* tids, const unsigned long long* tv, int* keep, hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(k_keep_new, dim3(div_up(n, kCcdBlock)), dim3(kCcdBlock), 0, s, n, ee, order, pairs, toc, qids,
                       tids, tv, keep);
}

void launch_keep_current(int lo, int hi, const double* gam, double gmin, int* keep, hipStream_t s) {
  if (hi > lo)
    hipLaunchKernelGGL(k_keep_current, dim3(div_up(hi - lo, kCcdBlock)), dim3(kCcdBlock), 0, s, lo, hi, gam, gmin,
                       keep);
}

void launch_scatter_current(int lo, int hi, const int* keep, const int* pos, int base, const int4* ids,
                            const double* lam, const double* gam, int4* oids, double* olam, double* ogam,
                            hipStream_t s) {
  if (hi > lo)
    hipLaunchKernelGGL(k_scatter_current, dim3(div_up(hi - lo, kCcdBlock)), dim3(kCcdBlock), 0, s, lo, hi, keep, pos,
                       base, ids, lam, gam, oids, olam, ogam);
}

void launch_scatter_new(int n, bool ee, const int* keep, const int* pos, int base, const int* order,
                        const int2* pairs, const int* qids, const int* tids, int4* oids, double* olam, double* ogam,
                        hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(k_scatter_new, dim3(div_up(n, kCcdBlock)), dim3(kCcdBlock), 0, s, n, ee, keep, pos, base,
                       order, pairs, qids, tids, oids, olam, ogam);
}

int ccd_min_parts(int n) { return std::max(1, std::min(div_up(n, kCcdBlock), 256)); }

void launch_min_toc(int n, const double* toc, double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_min_toc, dim3(ccd_min_parts(n)), dim3(kCcdBlock), 0, s, n, toc, part);
}

int inversion_parts(int T) { return std::max(1, div_up(T, kCcdBlock)); }

void launch_inversion_bound(int T, const int4* tets, const double* x, const double* xh, double sep, double* part,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_inversion_bound, dim3(inversion_parts(T)), dim3(kCcdBlock), 0, s, T, tets, x, xh, sep, part);
}

}  // namespace bfal
