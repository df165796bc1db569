// Host side of the collision queries: the surface of the mesh (once per
// problem), the two BVHs per call, the point-triangle and edge-edge queries
// with their narrow phase, and the two entry points built on them,
// bf_update_active_set (Algorithm 3) and bf_max_step_size (Algorithm 1).
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <utility>
#include <vector>

#include "problem.h"

namespace bfal {

namespace {

constexpr double kGammaRemove = 0.01;   // Algorithm 3: constraints whose decay factor fell below this go

// Boundary triangles (faces of exactly one tet, vertices ascending, rows
// sorted), their edges (ascending pairs, sorted) and vertices (sorted), built
// on the host from the tets and uploaded once.
bf_status ensure_surface(bf_problem* pb) {
  if (pb->surf_ready) return BF_OK;
  bf_context* c = pb->ctx;
  hipStream_t s = c->stream;
  const int T = pb->T;
  std::vector<int> tets(4LL * T);
  HIPCHK(c, hipMemcpyAsync(tets.data(), pb->tets.p, 16LL * T, hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  std::vector<std::array<int, 3>> faces;
  faces.reserve(4LL * T);
  const int fv[4][3] = {{0, 1, 2}, {0, 1, 3}, {0, 2, 3}, {1, 2, 3}};
  for (long long e = 0; e < T; ++e)
    for (auto& f : fv) {
      std::array<int, 3> a = {tets[4 * e + f[0]], tets[4 * e + f[1]], tets[4 * e + f[2]]};
      std::sort(a.begin(), a.end());
      faces.push_back(a);
    }
  std::sort(faces.begin(), faces.end());
  std::vector<int> tris;
  for (size_t i = 0; i < faces.size();) {
    size_t j = i + 1;
    while (j < faces.size() && faces[j] == faces[i]) ++j;
    if (j - i == 1) tris.insert(tris.end(), faces[i].begin(), faces[i].end());
    i = j;
  }
  const int nF = (int)(tris.size() / 3);
  std::vector<std::pair<int, int>> ev;
  ev.reserve(3LL * nF);
  std::vector<char> on(pb->N, 0);
  for (int f = 0; f < nF; ++f) {
    const int a = tris[3 * f], b = tris[3 * f + 1], d = tris[3 * f + 2];
    ev.push_back({a, b});
    ev.push_back({b, d});
    ev.push_back({a, d});
    on[a] = on[b] = on[d] = 1;
  }
  std::sort(ev.begin(), ev.end());
  ev.erase(std::unique(ev.begin(), ev.end()), ev.end());
  std::vector<int> edges;
  edges.reserve(2 * ev.size());
  for (auto& p : ev) {
    edges.push_back(p.first);
    edges.push_back(p.second);
  }
  std::vector<int> verts;
  for (int v = 0; v < pb->N; ++v)
    if (on[v]) verts.push_back(v);
  pb->nF = nF;
  pb->nE = (int)ev.size();
  pb->nV = (int)verts.size();
  ALLOC(c, pb->stris, 12LL * nF + 16);
  ALLOC(c, pb->sedges, 8LL * pb->nE + 16);
  ALLOC(c, pb->sverts, 4LL * pb->nV + 16);
  if (nF) HIPCHK(c, hipMemcpyAsync(pb->stris.p, tris.data(), 12LL * nF, hipMemcpyHostToDevice, s));
  if (pb->nE) HIPCHK(c, hipMemcpyAsync(pb->sedges.p, edges.data(), 8LL * pb->nE, hipMemcpyHostToDevice, s));
  if (pb->nV) HIPCHK(c, hipMemcpyAsync(pb->sverts.p, verts.data(), 4LL * pb->nV, hipMemcpyHostToDevice, s));
  HIPCHK(c, hipStreamSynchronize(s));
  pb->surf_ready = true;
  return BF_OK;
}

bf_status ensure_sort_tmp(bf_problem* pb, int n) {
  bf_context* c = pb->ctx;
  const size_t need = std::max(ccd_sort_tmp_bytes(std::max(n, 1)), ccd_sort_keys_tmp_bytes(std::max(n, 1)));
  ALLOC(c, pb->sort_tmp, need);
  return BF_OK;
}

// A BVH over n primitives of k vertices (ids AoS [n][k]).
bf_status build_tree(bf_problem* pb, int n, const int* ids, int k, const double* xh, DevBuf& box, DevBuf& key,
                     DevBuf& key2, DevBuf& child, DevBuf& parent, DevBuf& node, DevBuf& arrive) {
  // parent holds the internal nodes' leaf ranges, arrive the sparse table of run boxes
  bf_context* c = pb->ctx;
  hipStream_t s = c->stream;
  if (n == 0) return BF_OK;
  ALLOC(c, box, 24LL * n);
  ALLOC(c, key, 8LL * n);
  ALLOC(c, key2, 8LL * n);
  ALLOC(c, child, 8LL * std::max(n - 1, 1));
  ALLOC(c, parent, 8LL * std::max(n - 1, 1));          // internal node leaf ranges
  ALLOC(c, node, 48LL * n);
  ALLOC(c, arrive, 24LL * n * ccd_table_levels(n));    // sparse table of run boxes
  ALLOC(c, pb->bpart, 24LL * ccd_bounds_parts(n));
  launch_prim_boxes(n, ids, k, pb->x.as<double>(), xh, box.p, s);
  launch_morton(n, box.p, pb->bpart.p, key.as<unsigned long long>(), s);
  bf_status st = ensure_sort_tmp(pb, n);
  if (st != BF_OK) return st;
  HIPCHK(c, ccd_sort_keys(pb->sort_tmp.p, pb->sort_tmp.bytes, key.as<unsigned long long>(),
                          key2.as<unsigned long long>(), n, s));
  launch_build_tree(n, key2.as<unsigned long long>(), box.p, child.as<int2>(), parent.as<int2>(), node.p, arrive.p,
                    s);
  return BF_OK;
}

struct Collide {
  int hits[2] = {0, 0};
  long long cand[2] = {0, 0};
  float ms_tree = 0.f, ms_query = 0.f;
};

// Both BVHs and both queries along x -> xh: the colliding pairs of each kind
// (query index, tree index) with their times in qpairs / qtoc.
bf_status collide(bf_problem* pb, const double* xh, double sep, Collide& out) {
  bf_context* c = pb->ctx;
  hipStream_t s = c->stream;
  bf_status st = ensure_surface(pb);
  if (st != BF_OK) return st;
  HIPCHK(c, hipEventRecord(pb->ev[0], s));
  st = build_tree(pb, pb->nF, pb->stris.as<int>(), 3, xh, pb->tbox, pb->tkey, pb->tkey2, pb->tchild, pb->tparent,
                  pb->tnode, pb->tarrive);
  if (st != BF_OK) return st;
  st = build_tree(pb, pb->nE, pb->sedges.as<int>(), 2, xh, pb->ebox, pb->ekey, pb->ekey2, pb->echild, pb->eparent,
                  pb->enode, pb->earrive);
  if (st != BF_OK) return st;
  HIPCHK(c, hipEventRecord(pb->ev[1], s));
  ALLOC(c, pb->qcount, 4 * 32);
  int* cnt = pb->qcount.as<int>();
  bool todo[2] = {true, true};
  for (int round = 0; round < 2 && (todo[0] || todo[1]); ++round) {
    for (int kind = 0; kind < 2; ++kind) {
      if (!todo[kind]) continue;
      const int nq = kind ? pb->nE : pb->nV;
      if (pb->qcap[kind] == 0) pb->qcap[kind] = std::max(4096, 4 * nq);
      ALLOC(c, pb->qpairs[kind], 8LL * pb->qcap[kind]);
      ALLOC(c, pb->qtoc[kind], 8LL * pb->qcap[kind]);
      HIPCHK(c, hipMemsetAsync(cnt + 8 * kind, 0, 32, s));
      if (kind == 0)
        launch_query(false, pb->nV, pb->sverts.as<int>(), pb->nF, pb->stris.as<int>(), pb->tchild.as<int2>(),
                     pb->tnode.p, pb->tkey2.as<unsigned long long>(), pb->x.as<double>(), xh, pb->delta, sep,
                     cnt, pb->qcap[0], pb->qpairs[0].as<int2>(), pb->qtoc[0].as<double>(), s);
      else
        launch_query(true, pb->nE, pb->sedges.as<int>(), pb->nE, pb->sedges.as<int>(), pb->echild.as<int2>(),
                     pb->enode.p, pb->ekey2.as<unsigned long long>(), pb->x.as<double>(), xh, pb->delta, sep,
                     cnt + 8, pb->qcap[1], pb->qpairs[1].as<int2>(), pb->qtoc[1].as<double>(), s);
    }
    int h[16];
    HIPCHK(c, hipMemcpyAsync(h, cnt, sizeof(h), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    for (int kind = 0; kind < 2; ++kind) {
      if (!todo[kind]) continue;
      if (h[8 * kind + 1]) return fail(c, BF_ERR_HIP, "BVH traversal stack overflow");
      long long cand = 0;
      std::memcpy(&cand, h + 8 * kind + 2, sizeof(cand));
      out.cand[kind] = cand;
      out.hits[kind] = h[8 * kind];
      if (h[8 * kind] > pb->qcap[kind]) {
        pb->qcap[kind] = h[8 * kind] + h[8 * kind] / 4 + 1024;   // run this kind again with room for every pair
      } else {
        todo[kind] = false;
      }
    }
  }
  if (todo[0] || todo[1]) return fail(c, BF_ERR_HIP, "collision pair buffer did not settle");
  pb->qhits[0] = out.hits[0];
  pb->qhits[1] = out.hits[1];
  pb->collided = true;
  HIPCHK(c, hipEventRecord(pb->ev[2], s));
  HIPCHK(c, hipEventSynchronize(pb->ev[2]));
  (void)hipEventElapsedTime(&out.ms_tree, pb->ev[0], pb->ev[1]);
  (void)hipEventElapsedTime(&out.ms_query, pb->ev[1], pb->ev[2]);
  return BF_OK;
}

// The x_hat a collision call uses: the problem's own, or a caller's array
// copied to the device.
bf_status resolve_xhat(bf_problem* pb, const double* x_hat, int32_t mem, const double** out) {
  bf_context* c = pb->ctx;
  if (!x_hat) {
    *out = pb->xh.as<double>();
    return BF_OK;
  }
  if (mem != BF_MEM_HOST && mem != BF_MEM_DEVICE) return fail(c, BF_ERR_INVALID_ARG, "bad mem kind");
  ALLOC(c, pb->xq, 24LL * pb->N);
  HIPCHK(c, hipMemcpyAsync(pb->xq.p, x_hat, 24LL * pb->N, kind_in(mem), c->stream));
  *out = pb->xq.as<double>();
  return BF_OK;
}

bf_status check_ccd_args(bf_problem* pb, double sep) {
  bf_context* c = pb->ctx;
  if (!pb->has_state) return fail(c, BF_ERR_STATE, "bf_set_state must be called first");
  if (pb->cap_nnzb == 0) return fail(c, BF_ERR_STATE, "bf_set_constraints must be called first (kappa, delta)");
  if (!(sep > 0.0 && sep < 1.0)) return fail(c, BF_ERR_INVALID_ARG, "sep must lie in (0, 1)");
  return BF_OK;
}

}  // namespace

}  // namespace bfal

using namespace bfal;

extern "C" {

bf_status bf_max_step_size(bf_problem* pb, const double* x_hat, int32_t mem, double sep, double* alpha,
                           bf_ccd_stats* stats) {
  if (!pb) return BF_ERR_INVALID_ARG;
  bf_context* c = pb->ctx;
  if (!alpha) return fail(c, BF_ERR_INVALID_ARG, "alpha is NULL");
  if (sep == 0.0) sep = 0.1;
  bf_status st = check_ccd_args(pb, sep);
  if (st != BF_OK) return st;
  HIPCHK(c, hipSetDevice(c->device));
  hipStream_t s = c->stream;
  const double* xh = nullptr;
  st = resolve_xhat(pb, x_hat, mem, &xh);
  if (st != BF_OK) return st;
  Collide col;
  st = collide(pb, xh, sep, col);
  if (st != BF_OK) return st;
  const int m0 = ccd_min_parts(col.hits[0]), m1 = ccd_min_parts(col.hits[1]), mi = inversion_parts(pb->T);
  ALLOC(c, pb->mpart, 8LL * (m0 + m1 + mi));
  double* mp = pb->mpart.as<double>();
  launch_min_toc(col.hits[0], pb->qtoc[0].as<double>(), mp, s);
  launch_min_toc(col.hits[1], pb->qtoc[1].as<double>(), mp + m0, s);
  launch_inversion_bound(pb->T, pb->tets.as<int4>(), pb->x.as<double>(), xh, sep, mp + m0 + m1, s);
  std::vector<double> h(m0 + m1 + mi);
  HIPCHK(c, hipMemcpyAsync(h.data(), mp, 8LL * h.size(), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  double a_ccd = 1.0, a_inv = 1.0;
  for (int k = 0; k < m0 + m1; ++k) a_ccd = std::min(a_ccd, h[k]);
  for (int k = 0; k < mi; ++k) a_inv = std::min(a_inv, h[m0 + m1 + k]);
  *alpha = std::min(a_ccd, a_inv);
  if (stats) {
    *stats = bf_ccd_stats{};
    stats->candidates_pt = col.cand[0];
    stats->candidates_ee = col.cand[1];
    stats->colliding_pt = col.hits[0];
    stats->colliding_ee = col.hits[1];
    stats->n_pt = pb->n_pt;
    stats->n_ee = pb->n_ee;
    stats->alpha_ccd = a_ccd;
    stats->alpha_inversion = a_inv;
    stats->ms_tree = col.ms_tree;
    stats->ms_query = col.ms_query;
  }
  c->err.clear();
  return BF_OK;
}

bf_status bf_update_active_set(bf_problem* pb, const double* x_hat, int32_t mem, double sep, bf_ccd_stats* stats) {
  if (!pb) return BF_ERR_INVALID_ARG;
  bf_context* c = pb->ctx;
  if (sep == 0.0) sep = 0.1;
  bf_status st = check_ccd_args(pb, sep);
  if (st != BF_OK) return st;
  HIPCHK(c, hipSetDevice(c->device));
  hipStream_t s = c->stream;
  const double* xh = nullptr;
  st = resolve_xhat(pb, x_hat, mem, &xh);
  if (st != BF_OK) return st;
  Collide col;
  st = collide(pb, xh, sep, col);
  if (st != BF_OK) return st;
  HIPCHK(c, hipEventRecord(pb->ev[0], s));
  const int n0 = col.hits[0], n1 = col.hits[1], nh = n0 + n1;
  const int n_pt = pb->n_pt, n_c = pb->n_c;
  // canonical order of the colliding pairs of each kind
  ALLOC(c, pb->pkey, 8LL * nh + 8);
  ALLOC(c, pb->pkey2, 8LL * nh + 8);
  ALLOC(c, pb->pidx, 4LL * nh + 4);
  ALLOC(c, pb->pidx2, 4LL * nh + 4);
  st = ensure_sort_tmp(pb, std::max(n0, n1));
  if (st != BF_OK) return st;
  int* order[2] = {pb->pidx2.as<int>(), pb->pidx2.as<int>() + n0};
  for (int kind = 0; kind < 2; ++kind) {
    const int n = kind ? n1 : n0, off = kind ? n0 : 0;
    if (!n) continue;
    launch_pair_keys(n, pb->qpairs[kind].as<int2>(), pb->pkey.as<unsigned long long>() + off,
                     pb->pidx.as<int>() + off, s);
    HIPCHK(c, ccd_sort_pairs(pb->sort_tmp.p, pb->sort_tmp.bytes, pb->pkey.as<unsigned long long>() + off,
                             pb->pkey2.as<unsigned long long>() + off, pb->pidx.as<int>() + off, order[kind], n, s));
  }
  // the current constraints in a hash set (keyed by their canonical ids)
  int* table = nullptr;
  unsigned int mask = 0;
  if (n_c > 0) {
    unsigned int size = 64;
    while (size < 2u * (unsigned int)n_c + 1u) size <<= 1;
    mask = size - 1;
    ALLOC(c, pb->htable, 4LL * size);
    table = pb->htable.as<int>();
    fill_int(table, -1, size, s);
    launch_hash_insert(n_c, n_pt, pb->cids.as<int4>(), table, mask, s);
  }
  // new pairs and the per-vertex earliest time over them (PT and EE together)
  ALLOC(c, pb->tvmin, 8LL * pb->N);
  launch_fill_u64(pb->tvmin.as<unsigned long long>(), 0x7FF0000000000000ull, pb->N, s);
  const long long nmax = std::max({(long long)n0, (long long)n1, (long long)n_c, 1LL});
  ALLOC(c, pb->ctmp, 4LL * scan_tmp_ints(nmax) + 16);
  ALLOC(c, pb->keepc, 4LL * n_c + 4);
  ALLOC(c, pb->posc, 4LL * n_c + 4);
  int* tot = pb->qcount.as<int>() + 16;   // [0..1] new, [2..3] kept new, [4..5] kept current
  HIPCHK(c, hipMemsetAsync(tot, 0, 32, s));
  const int* qids[2] = {pb->sverts.as<int>(), pb->sedges.as<int>()};
  const int* tids[2] = {pb->stris.as<int>(), pb->sedges.as<int>()};
  for (int kind = 0; kind < 2; ++kind) {
    const int n = kind ? n1 : n0;
    ALLOC(c, pb->keepn[kind], 4LL * n + 4);
    ALLOC(c, pb->posn[kind], 4LL * n + 4);
    if (!n) continue;
    launch_new_and_tv(n, kind == 1, order[kind], pb->qpairs[kind].as<int2>(), pb->qtoc[kind].as<double>(),
                      qids[kind], tids[kind], n_pt, pb->cids.as<int4>(), table, mask, pb->x.as<double>(),
                      pb->keepn[kind].as<int>(), pb->tvmin.as<unsigned long long>(), s);
    scan_exclusive(pb->keepn[kind].as<int>(), pb->posn[kind].as<int>(), n, tot + kind, pb->ctmp.as<int>(), s);
  }
  for (int kind = 0; kind < 2; ++kind) {
    const int n = kind ? n1 : n0;
    if (!n) continue;
    launch_keep_new(n, kind == 1, order[kind], pb->qpairs[kind].as<int2>(), pb->qtoc[kind].as<double>(), qids[kind],
                    tids[kind], pb->tvmin.as<unsigned long long>(), pb->keepn[kind].as<int>(), s);
    scan_exclusive(pb->keepn[kind].as<int>(), pb->posn[kind].as<int>(), n, tot + 2 + kind, pb->ctmp.as<int>(), s);
  }
  // surviving current constraints (gamma >= 0.01), PT part then EE part
  const int lo[2] = {0, n_pt}, hi[2] = {n_pt, n_c};
  for (int kind = 0; kind < 2; ++kind) {
    if (hi[kind] <= lo[kind]) continue;
    launch_keep_current(lo[kind], hi[kind], pb->cgam.as<double>(), kGammaRemove, pb->keepc.as<int>() + lo[kind], s);
    scan_exclusive(pb->keepc.as<int>() + lo[kind], pb->posc.as<int>() + lo[kind], hi[kind] - lo[kind], tot + 4 + kind,
                   pb->ctmp.as<int>(), s);
  }
  int h[6];
  HIPCHK(c, hipMemcpyAsync(h, tot, sizeof(h), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  const int new_pt = h[0], new_ee = h[1], add_pt = h[2], add_ee = h[3], kc_pt = h[4], kc_ee = h[5];
  const int npt2 = kc_pt + add_pt, nee2 = kc_ee + add_ee, n2 = npt2 + nee2;
  if ((long long)n2 * 10 >= (1LL << 31)) return fail(c, BF_ERR_INVALID_ARG, "too many constraints after the update");
  ALLOC(c, pb->nids, 16LL * n2 + 16);
  ALLOC(c, pb->nlam, 8LL * n2 + 8);
  ALLOC(c, pb->ngam, 8LL * n2 + 8);
  int4* oids = pb->nids.as<int4>();
  double* olam = pb->nlam.as<double>();
  double* ogam = pb->ngam.as<double>();
  const int base_cur[2] = {0, npt2}, base_new[2] = {kc_pt, npt2 + kc_ee};
  for (int kind = 0; kind < 2; ++kind) {
    if (hi[kind] > lo[kind])
      launch_scatter_current(lo[kind], hi[kind], pb->keepc.as<int>() + lo[kind], pb->posc.as<int>() + lo[kind],
                             base_cur[kind], pb->cids.as<int4>(), pb->clam.as<double>(), pb->cgam.as<double>(), oids,
                             olam, ogam, s);
    const int n = kind ? n1 : n0;
    if (n)
      launch_scatter_new(n, kind == 1, pb->keepn[kind].as<int>(), pb->posn[kind].as<int>(), base_new[kind],
                         order[kind], pb->qpairs[kind].as<int2>(), qids[kind], tids[kind], oids, olam, ogam, s);
  }
  HIPCHK(c, hipEventRecord(pb->ev[1], s));
  HIPCHK(c, hipStreamSynchronize(s));
  std::swap(pb->cids, pb->nids);
  std::swap(pb->clam, pb->nlam);
  std::swap(pb->cgam, pb->ngam);
  st = size_constraint_buffers(pb, npt2, nee2);
  if (st != BF_OK) return st;
  pb->stepped = false;   // the linearization of the old set no longer applies
  if (stats) {
    float ms_upd = 0.f;
    (void)hipEventElapsedTime(&ms_upd, pb->ev[0], pb->ev[1]);
    *stats = bf_ccd_stats{};
    stats->candidates_pt = col.cand[0];
    stats->candidates_ee = col.cand[1];
    stats->colliding_pt = n0;
    stats->colliding_ee = n1;
    stats->new_pt = new_pt;
    stats->new_ee = new_ee;
    stats->added_pt = add_pt;
    stats->added_ee = add_ee;
    stats->removed = n_c - kc_pt - kc_ee;
    stats->n_pt = npt2;
    stats->n_ee = nee2;
    stats->alpha_ccd = 1.0;
    stats->alpha_inversion = 1.0;
    stats->ms_tree = col.ms_tree;
    stats->ms_query = col.ms_query;
    stats->ms_update = ms_upd;
  }
  c->err.clear();
  return BF_OK;
}

bf_status bf_get_collisions(bf_problem* pb, int32_t* pt, double* pt_toc, int32_t* ee, double* ee_toc) {
  if (!pb) return BF_ERR_INVALID_ARG;
  bf_context* c = pb->ctx;
  if (!pb->collided) return fail(c, BF_ERR_STATE, "no collision call has been made");
  hipStream_t s = c->stream;
  const int n = std::max(pb->qhits[0], pb->qhits[1]);
  ALLOC(c, pb->nids, 16LL * n + 16);
  int32_t* rows[2] = {pt, ee};
  double* tocs[2] = {pt_toc, ee_toc};
  const int* qids[2] = {pb->sverts.as<int>(), pb->sedges.as<int>()};
  const int* tids[2] = {pb->stris.as<int>(), pb->sedges.as<int>()};
  for (int kind = 0; kind < 2; ++kind) {
    const int m = pb->qhits[kind];
    if (!m) continue;
    if (rows[kind]) {
      launch_pair_rows(m, kind == 1, pb->qpairs[kind].as<int2>(), qids[kind], tids[kind], pb->nids.as<int4>(), s);
      HIPCHK(c, hipMemcpyAsync(rows[kind], pb->nids.p, 16LL * m, hipMemcpyDeviceToHost, s));
      HIPCHK(c, hipStreamSynchronize(s));
    }
    if (tocs[kind]) HIPCHK(c, hipMemcpyAsync(tocs[kind], pb->qtoc[kind].p, 8LL * m, hipMemcpyDeviceToHost, s));
  }
  HIPCHK(c, hipStreamSynchronize(s));
  return BF_OK;
}

bf_status bf_get_constraint_counts(bf_problem* pb, int32_t* n_pt, int32_t* n_ee) {
  if (!pb) return BF_ERR_INVALID_ARG;
  if (!n_pt || !n_ee) return fail(pb->ctx, BF_ERR_INVALID_ARG, "count pointer is NULL");
  *n_pt = pb->n_pt;
  *n_ee = pb->n_ee;
  return BF_OK;
}

bf_status bf_get_constraints(bf_problem* pb, int32_t* pt, int32_t* ee, double* lambda, double* gamma, int32_t mem) {
  if (!pb) return BF_ERR_INVALID_ARG;
  bf_context* c = pb->ctx;
  if (mem != BF_MEM_HOST && mem != BF_MEM_DEVICE) return fail(c, BF_ERR_INVALID_ARG, "bad mem kind");
  hipStream_t s = c->stream;
  const hipMemcpyKind k = kind_out(mem);
  if (pt && pb->n_pt) HIPCHK(c, hipMemcpyAsync(pt, pb->cids.p, 16LL * pb->n_pt, k, s));
  if (ee && pb->n_ee) HIPCHK(c, hipMemcpyAsync(ee, pb->cids.as<char>() + 16LL * pb->n_pt, 16LL * pb->n_ee, k, s));
  if (lambda && pb->n_c) HIPCHK(c, hipMemcpyAsync(lambda, pb->clam.p, 8LL * pb->n_c, k, s));
  if (gamma && pb->n_c) HIPCHK(c, hipMemcpyAsync(gamma, pb->cgam.p, 8LL * pb->n_c, k, s));
  HIPCHK(c, hipStreamSynchronize(s));
  return BF_OK;
}

}  // extern "C"
