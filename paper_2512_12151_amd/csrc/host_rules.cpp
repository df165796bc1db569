// Host rules of libbfal (include/bfal_host.h): argument validation, the
// penalty stall rule of Section 5.2, the serving admission policy and the
// SpMV's slice plan.  Plain C++ without HIP, built with the host compiler, so
// the same object serves the library and a CPU-only (sanitizer) build.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <new>
#include <vector>

#include "../../include/bfal_host.h"

namespace {

bf_status reject(bf_status st, char* msg, int32_t cap, const char* text) {
  if (msg && cap > 0) std::snprintf(msg, (size_t)cap, "%s", text);
  return st;
}

bool finite_all(const double* a, long long n) {
  for (long long i = 0; i < n; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

bool distinct4(const int32_t* t) {
  return t[0] != t[1] && t[0] != t[2] && t[0] != t[3] && t[1] != t[2] && t[1] != t[3] && t[2] != t[3];
}

}  // namespace

struct bf_admission {
  struct Item {
    int64_t id;
    uint64_t footprint;
  };
  uint64_t budget = 0, used = 0;
  std::deque<Item> queue;
  std::vector<uint64_t> slot_bytes;   // footprint admitted into each slot
  std::vector<char> slot_used;
  std::vector<int32_t> free_slots;    // stack: the lowest slot index is reused first
};

extern "C" {

bf_status bf_check_mesh(const bf_mesh_desc* m, char* msg, int32_t cap) {
  if (!m || !m->tets || !m->rest || !m->E || !m->nu || !m->rho)
    return reject(BF_ERR_INVALID_ARG, msg, cap, "mesh descriptor or one of its arrays is NULL");
  if (m->n_nodes <= 0 || m->n_tets <= 0)
    return reject(BF_ERR_INVALID_ARG, msg, cap, "n_nodes and n_tets must be positive");
  if ((long long)m->n_tets * 10 >= (1LL << 31) || (long long)m->n_nodes * 3 >= (1LL << 31))
    return reject(BF_ERR_INVALID_ARG, msg, cap, "mesh too large for 32-bit slot indices");
  const int32_t N = m->n_nodes;
  for (long long e = 0; e < m->n_tets; ++e) {
    const int32_t* t = m->tets + 4 * e;
    for (int a = 0; a < 4; ++a)
      if (t[a] < 0 || t[a] >= N) return reject(BF_ERR_INVALID_ARG, msg, cap, "tet vertex index out of range");
    if (!distinct4(t)) return reject(BF_ERR_INVALID_ARG, msg, cap, "tet with a repeated vertex");
    if (!(m->E[e] > 0.0) || !std::isfinite(m->E[e]) || !(m->nu[e] > -1.0 && m->nu[e] < 0.5) ||
        !(m->rho[e] > 0.0) || !std::isfinite(m->rho[e]))
      return reject(BF_ERR_INVALID_ARG, msg, cap, "invalid material value");
    if (m->material && (m->material[e] < 0 || m->material[e] > 2))
      return reject(BF_ERR_INVALID_ARG, msg, cap,
                    "material code must be 0 (Neo-Hookean), 1 (stable Neo-Hookean) or 2 (corotated linear)");
  }
  if (!finite_all(m->rest, 3LL * N)) return reject(BF_ERR_INVALID_ARG, msg, cap, "non-finite rest position");
  return BF_OK;
}

bf_status bf_check_state(int32_t n_nodes, const double* x, const double* x_hat, const double* x_tilde, double dt,
                         char* msg, int32_t cap) {
  if (!x || !x_hat || !x_tilde) return reject(BF_ERR_INVALID_ARG, msg, cap, "state array is NULL");
  if (n_nodes <= 0) return reject(BF_ERR_INVALID_ARG, msg, cap, "n_nodes must be positive");
  if (!(dt > 0.0) || !std::isfinite(dt)) return reject(BF_ERR_INVALID_ARG, msg, cap, "dt must be positive and finite");
  const long long n3 = 3LL * n_nodes;
  if (!finite_all(x, n3) || !finite_all(x_hat, n3) || !finite_all(x_tilde, n3))
    return reject(BF_ERR_INVALID_ARG, msg, cap, "non-finite state value");
  return BF_OK;
}

bf_status bf_check_constraints(int32_t n_nodes, const bf_constraint_desc* cd, char* msg, int32_t cap) {
  if (!cd) return reject(BF_ERR_INVALID_ARG, msg, cap, "constraint descriptor is NULL");
  if (cd->n_pt < 0 || cd->n_ee < 0) return reject(BF_ERR_INVALID_ARG, msg, cap, "negative constraint count");
  const long long nc = (long long)cd->n_pt + cd->n_ee;
  if (nc * 10 >= (1LL << 31)) return reject(BF_ERR_INVALID_ARG, msg, cap, "too many constraints");
  if ((cd->n_pt && !cd->pt) || (cd->n_ee && !cd->ee) || (nc && !cd->lambda))
    return reject(BF_ERR_INVALID_ARG, msg, cap, "constraint array is NULL");
  if (!(cd->kappa > 0.0) || !std::isfinite(cd->kappa))
    return reject(BF_ERR_INVALID_ARG, msg, cap, "kappa must be positive");
  if (!(cd->delta >= 0.0) || !std::isfinite(cd->delta))
    return reject(BF_ERR_INVALID_ARG, msg, cap, "delta must be >= 0");
  for (int part = 0; part < 2; ++part) {
    const int32_t* a = part ? cd->ee : cd->pt;
    const long long n = part ? cd->n_ee : cd->n_pt;
    for (long long i = 0; i < n; ++i) {
      const int32_t* t = a + 4 * i;
      for (int k = 0; k < 4; ++k)
        if (t[k] < 0 || t[k] >= n_nodes)
          return reject(BF_ERR_INVALID_ARG, msg, cap, "constraint vertex index out of range");
      if (!distinct4(t)) return reject(BF_ERR_DEGENERATE_CONSTRAINT, msg, cap, "constraint with a repeated vertex");
    }
  }
  for (long long i = 0; i < nc; ++i) {
    if (!(cd->lambda[i] >= 0.0) || !std::isfinite(cd->lambda[i]))
      return reject(BF_ERR_INVALID_ARG, msg, cap, "lambda must be finite and >= 0");
    if (cd->gamma && !(cd->gamma[i] > 0.0 && cd->gamma[i] <= 1.0))
      return reject(BF_ERR_INVALID_ARG, msg, cap, "gamma must lie in (0, 1]");
  }
  return BF_OK;
}

bf_status bf_check_solve_opts(const bf_solve_opts* o, char* msg, int32_t cap) {
  if (!o) return reject(BF_ERR_INVALID_ARG, msg, cap, "opts is NULL");
  if (!(o->tol > 0.0) || o->max_iter < 0)
    return reject(BF_ERR_INVALID_ARG, msg, cap, "tol must be > 0 and max_iter >= 0");
  if (o->precision != BF_PREC_FP32 && o->precision != BF_PREC_BF16_REFINE)
    return reject(BF_ERR_INVALID_ARG, msg, cap, "unsupported precision mode");
  if (o->precision == BF_PREC_BF16_REFINE && !(o->refine_tol > 0.0))
    return reject(BF_ERR_INVALID_ARG, msg, cap, "refine_tol must be > 0");
  return BF_OK;
}

int32_t bf_stall_step(bf_stall_rule* r, double alpha, double* kappa, double* delta) {
  if (!r || !kappa || !delta || r->window < 1) return -1;
  r->count = alpha < r->alpha_min ? r->count + 1 : 0;
  if (r->count < r->window) return 0;
  *kappa *= 2.0;
  *delta *= 0.5;
  r->count = 0;
  return 1;
}

bf_status bf_admission_create(uint64_t hbm_budget, int32_t slots, bf_admission** out) {
  if (!out || hbm_budget == 0 || slots < 1) return BF_ERR_INVALID_ARG;
  *out = nullptr;
  bf_admission* a = new (std::nothrow) bf_admission();
  if (!a) return BF_ERR_OOM;
  try {
    a->budget = hbm_budget;
    a->slot_bytes.assign(slots, 0);
    a->slot_used.assign(slots, 0);
    for (int32_t i = slots - 1; i >= 0; --i) a->free_slots.push_back(i);
  } catch (...) {
    delete a;
    return BF_ERR_OOM;
  }
  *out = a;
  return BF_OK;
}

void bf_admission_destroy(bf_admission* a) { delete a; }

bf_status bf_admission_push(bf_admission* a, int64_t id, uint64_t footprint) {
  if (!a) return BF_ERR_INVALID_ARG;
  try {
    a->queue.push_back({id, footprint});
  } catch (...) {
    return BF_ERR_OOM;
  }
  return BF_OK;
}

int32_t bf_admission_next(bf_admission* a, int64_t* id, int32_t* slot) {
  if (!a || !id || !slot || a->queue.empty()) return 0;
  const bf_admission::Item h = a->queue.front();
  if (h.footprint > a->budget) {   // can never fit: reject without blocking the queue
    a->queue.pop_front();
    *id = h.id;
    *slot = -1;
    return -1;
  }
  if (a->free_slots.empty() || a->used + h.footprint > a->budget) return 0;
  a->queue.pop_front();
  const int32_t s = a->free_slots.back();
  a->free_slots.pop_back();
  a->slot_used[s] = 1;
  a->slot_bytes[s] = h.footprint;
  a->used += h.footprint;
  *id = h.id;
  *slot = s;
  return 1;
}

bf_status bf_admission_release(bf_admission* a, int32_t slot, uint64_t footprint) {
  if (!a || slot < 0 || slot >= (int32_t)a->slot_used.size() || !a->slot_used[slot] ||
      a->slot_bytes[slot] != footprint)
    return BF_ERR_INVALID_ARG;
  a->slot_used[slot] = 0;
  a->slot_bytes[slot] = 0;
  a->used -= footprint;
  a->free_slots.push_back(slot);
  return BF_OK;
}

bf_status bf_slice_plan(int32_t nslices, const int32_t* slot_u, const int32_t* slot_l, int32_t pairs,
                        int32_t nparts, int32_t* wave_ptr, int32_t* wave_slices) {
  if (!slot_u || !slot_l || !wave_ptr || !wave_slices || nslices < 1 || pairs < 1 || nparts < 8 || nparts % 8)
    return BF_ERR_INVALID_ARG;
  for (int32_t s = 0; s <= nslices; ++s)
    if (slot_u[s] % 64 || slot_l[s] % 64 || (s > 0 && (slot_u[s] < slot_u[s - 1] || slot_l[s] < slot_l[s - 1])))
      return BF_ERR_INVALID_ARG;
  const int32_t per_x = nparts / 8;
  std::vector<int64_t> load;
  std::vector<int32_t> cost, part_of, cur, blk;
  try {
    load.assign(nparts, 0);
    cost.resize(nslices);
    part_of.resize(nslices);
    cur.resize(nparts);
    blk.reserve(2 * (size_t)per_x);
  } catch (...) {
    return BF_ERR_OOM;
  }
  for (int32_t s = 0; s < nslices; ++s) {
    const int32_t wu = (slot_u[s + 1] - slot_u[s]) / 64, wl = (slot_l[s + 1] - slot_l[s]) / 64;
    const int32_t w = wu > wl ? wu : wl;
    cost[s] = (w + pairs - 1) / pairs + 1;
  }
  int64_t tot = 0;
  for (int32_t s = 0; s < nslices; ++s) tot += cost[s];
  // window x starts at the first slice whose cost prefix reaches x / 8 of the total
  int32_t start[9];
  start[0] = 0;
  int32_t x = 1;
  int64_t acc = 0;
  for (int32_t s = 0; s < nslices && x < 8; ++s) {
    while (x < 8 && 8 * acc >= x * tot) start[x++] = s;
    acc += cost[s];
  }
  while (x < 8) start[x++] = nslices;
  start[8] = nslices;
  // each window in blocks of two slices per part, taken in order; inside a
  // block the costliest slices go first (ties in slice order), each to the
  // part with the least cost so far
  const int32_t bsize = 2 * per_x;
  for (x = 0; x < 8; ++x) {
    int64_t* lx = load.data() + (int64_t)x * per_x;
    for (int32_t b0 = start[x]; b0 < start[x + 1]; b0 += bsize) {
      const int32_t b1 = std::min(start[x + 1], b0 + bsize);
      blk.clear();
      for (int32_t s = b0; s < b1; ++s) blk.push_back(s);
      std::stable_sort(blk.begin(), blk.end(), [&](int32_t a, int32_t b) { return cost[a] > cost[b]; });
      for (const int32_t s : blk) {
        int32_t best = 0;
        for (int32_t p = 1; p < per_x; ++p)
          if (lx[p] < lx[best]) best = p;
        lx[best] += cost[s];
        part_of[s] = x * per_x + best;
      }
    }
  }
  for (int32_t p = 0; p <= nparts; ++p) wave_ptr[p] = 0;
  for (int32_t s = 0; s < nslices; ++s) ++wave_ptr[part_of[s] + 1];
  for (int32_t p = 0; p < nparts; ++p) wave_ptr[p + 1] += wave_ptr[p];
  for (int32_t p = 0; p < nparts; ++p) cur[p] = wave_ptr[p];
  for (int32_t s = 0; s < nslices; ++s) wave_slices[cur[part_of[s]]++] = s;
  return BF_OK;
}

uint64_t bf_admission_used(const bf_admission* a) { return a ? a->used : 0; }

int32_t bf_admission_waiting(const bf_admission* a) { return a ? (int32_t)a->queue.size() : 0; }

int32_t bf_admission_active(const bf_admission* a) {
  if (!a) return 0;
  return (int32_t)(a->slot_used.size() - a->free_slots.size());
}

}  // extern "C"
