// Serving engine of libbfal: continuous batching of independent Newton-step
// solves (one request = one mesh with its state and active constraint set).
//
// Native threads share one device:
//   admission  (several workers, one stream each) take submitted requests in
//              arrival order, admit the head of the queue when its device
//              footprint fits the HBM budget and a slot is free, and run its
//              setup and assembly (per-mesh setup, constraint linearization,
//              merged pattern, element and contact blocks, block-Jacobi
//              factors, sliced storage) on the worker's stream;
//   batch      runs the PCG of every admitted request together: each round is
//              a few iterations of the batched SpMV/update kernel pair, whose
//              grid is the concatenation of the requests' grids (a
//              block-diagonal system with per-request scalars, so requests of
//              any size and at any iteration share a launch).  Between rounds
//              it reads every request's status with one small copy, retires
//              the finished ones (p = L^{-T} x, copy out, stats), frees their
//              budget and slot, and adds newly assembled requests.
// A request's device state stays resident in its slot from admission to
// retirement; slots (and their device buffers) are reused by later requests.
// With max_active = 1 the same engine serves one request at a time in arrival
// order, the baseline that batching is measured against.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "problem.h"

using namespace bfal;

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Request {
  int64_t id = 0;
  int32_t N = 0, T = 0, n_pt = 0, n_ee = 0;
  std::vector<int32_t> tets, pt, ee, material;
  std::vector<double> rest, E, nu, rho, x, xh, xt, lam, gam;
  std::vector<uint8_t> fixed;
  double dt = 0.0, kappa = 0.0, delta = 0.0;
  bf_solve_opts opts{};
  size_t footprint = 0;
  double t_submit = 0.0, t_admit = 0.0, t_done = 0.0, ms_setup = 0.0;
  // result
  std::vector<double> p;
  bf_step_stats stats{};
  bf_status status = BF_OK;
  std::string err;
};

struct Slot {
  bf_problem* pb = nullptr;
  Request* req = nullptr;
  PcgSystem S{};
};

}  // namespace

struct bf_server {
  std::vector<bf_context*> admit_ctx;   // own contexts: one stream per admission worker
  bf_context* batch_ctx = nullptr;
  bf_admission* adm = nullptr;              // arrival-order admission by footprint and slot (bfal_host.h)
  int max_active = 1, iters_per_round = 8;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request*> pending;               // submitted, not admitted (the admission queue's order)
  std::deque<int> ready;                      // slots assembled by the admission thread
  std::vector<Slot> slots;
  std::unordered_map<int64_t, Request*> done; // finished, result not yet taken
  std::vector<int64_t> done_unreported;
  bool stop = false;
  std::vector<std::thread> admit_threads;
  std::thread batch_thread;
  // batch thread only
  std::vector<int> active;
  DevBuf sys_dev, map_spmv, map_vec, status_dev;
  PcgSystem* h_sys = nullptr;
  int* h_map = nullptr;
  int* h_status = nullptr;
  int h_map_cap = 0, h_sys_cap = 0;
};

namespace {

constexpr int kStatusInts = 4;   // per system: done, brk, iter, flags

__global__ void k_gather_status(const PcgSystem* __restrict__ sys, int n, int* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const PcgScalars* sc = sys[i].sc;
  out[kStatusInts * i] = sc->done;
  out[kStatusInts * i + 1] = sc->brk;
  out[kStatusInts * i + 2] = sc->iter;
  out[kStatusInts * i + 3] = sc->flags;
}

void finish_request(bf_server* sv, Request* r, bf_status st, const std::string& msg) {
  r->status = st;
  r->err = msg;
  r->t_done = now_s();
  std::lock_guard<std::mutex> lk(sv->mu);
  sv->done[r->id] = r;
  sv->done_unreported.push_back(r->id);
}

// Setup and assembly of one request in slot si, on an admission worker's stream.
bf_status prepare(bf_server* sv, bf_context* c, int si, Request* r) {
  Slot& sl = sv->slots[si];
  if (!sl.pb) {
    sl.pb = new (std::nothrow) bf_problem();
    if (!sl.pb) return fail(c, BF_ERR_OOM, "host allocation failed");
    sl.pb->ctx = c;
  }
  bf_problem* pb = sl.pb;
  pb->ctx = c;
  bf_mesh_desc m{r->N, r->T, r->tets.data(), r->rest.data(), r->E.data(), r->nu.data(), r->rho.data(),
                 r->fixed.empty() ? nullptr : r->fixed.data(), r->material.empty() ? nullptr : r->material.data()};
  bf_status st = problem_init(c, pb, &m, BF_MEM_HOST);
  if (st != BF_OK) return st;
  st = bf_set_state(pb, r->x.data(), r->xh.data(), r->xt.data(), r->dt, BF_MEM_HOST);
  if (st != BF_OK) return st;
  bf_constraint_desc cd{r->n_pt, r->n_ee, r->pt.empty() ? nullptr : r->pt.data(),
                        r->ee.empty() ? nullptr : r->ee.data(), r->lam.empty() ? nullptr : r->lam.data(),
                        r->gam.empty() ? nullptr : r->gam.data(), r->kappa, r->delta};
  st = bf_set_constraints(pb, &cd, BF_MEM_HOST);
  if (st != BF_OK) return st;
  st = step_assemble(pb, false);
  if (st != BF_OK) return st;
  sl.S = system_of(pb);
  launch_pcg_init(sl.S, pb->bhat.as<float>(), pb->bb_part.as<double>(), div_up(pb->N, kBlock), r->opts.tol,
                  r->opts.max_iter, r->opts.check_every, true, c->stream);
  int hf = 0;
  st = read_flags(pb, &hf);   // synchronizes the admission stream: the slot is complete
  if (st != BF_OK) return st;
  if (hf) return flags_to_status(c, hf);
  return BF_OK;
}

void admission_loop(bf_server* sv, int worker) {
  bf_context* c = sv->admit_ctx[worker];
  (void)hipSetDevice(c->device);
  for (;;) {
    Request* r = nullptr;
    int si = -1;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      for (;;) {
        if (sv->stop) return;
        int64_t id = 0;
        int32_t slot = -1;
        const int32_t d = bf_admission_next(sv->adm, &id, &slot);
        if (d == -1) {   // can never fit: rejected without blocking the queue
          Request* h = sv->pending.front();
          sv->pending.pop_front();
          lk.unlock();
          finish_request(sv, h, BF_ERR_BUDGET, "request footprint exceeds the server's HBM budget");
          lk.lock();
          continue;
        }
        if (d == 1) {
          r = sv->pending.front();
          sv->pending.pop_front();
          si = slot;
          break;
        }
        sv->cv.wait(lk);
      }
    }
    r->t_admit = now_s();
    const bf_status st = prepare(sv, c, si, r);
    r->ms_setup = (now_s() - r->t_admit) * 1e3;
    if (st != BF_OK) {
      const std::string msg = c->err;
      {
        std::lock_guard<std::mutex> lk(sv->mu);
        (void)bf_admission_release(sv->adm, si, r->footprint);
        sv->slots[si].req = nullptr;
      }
      finish_request(sv, r, st, msg);
      sv->cv.notify_all();
      continue;
    }
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      sv->slots[si].req = r;
      sv->ready.push_back(si);
    }
    sv->cv.notify_all();
  }
}

// Rebuild and upload the batch table: every active system gets its SpMV and
// update workgroups at consecutive offsets.
bf_status upload_table(bf_server* sv, int* nwg_spmv, int* nwg_vec) {
  bf_context* c = sv->batch_ctx;
  const int n = (int)sv->active.size();
  int ts = 0, tv = 0;
  for (int i : sv->active) {
    ts += sv->slots[i].S.spmv_nwg;
    tv += sv->slots[i].S.vec_nwg;
  }
  if (n > sv->h_sys_cap) {
    if (sv->h_sys) (void)hipHostFree(sv->h_sys);
    if (sv->h_status) (void)hipHostFree(sv->h_status);
    sv->h_sys = nullptr;
    sv->h_status = nullptr;
    HIPCHK(c, hipHostMalloc((void**)&sv->h_sys, sizeof(PcgSystem) * n, hipHostMallocDefault));
    HIPCHK(c, hipHostMalloc((void**)&sv->h_status, sizeof(int) * kStatusInts * n, hipHostMallocDefault));
    sv->h_sys_cap = n;
  }
  if (ts + tv > sv->h_map_cap) {
    if (sv->h_map) (void)hipHostFree(sv->h_map);
    sv->h_map = nullptr;
    HIPCHK(c, hipHostMalloc((void**)&sv->h_map, sizeof(int) * (ts + tv), hipHostMallocDefault));
    sv->h_map_cap = ts + tv;
  }
  int os = 0, ov = 0;
  for (int k = 0; k < n; ++k) {
    PcgSystem S = sv->slots[sv->active[k]].S;
    S.spmv_wg0 = os;
    S.vec_wg0 = ov;
    for (int b = 0; b < S.spmv_nwg; ++b) sv->h_map[os + b] = k;
    for (int b = 0; b < S.vec_nwg; ++b) sv->h_map[ts + ov + b] = k;
    os += S.spmv_nwg;
    ov += S.vec_nwg;
    sv->h_sys[k] = S;
  }
  // device tables grow geometrically (a reallocation frees the old buffer)
  const size_t want_sys = sizeof(PcgSystem) * std::max(n, 64);
  const size_t want_map = sizeof(int) * std::max(ts + tv, 4096);
  if (sv->sys_dev.bytes < sizeof(PcgSystem) * n) ALLOC(c, sv->sys_dev, 2 * want_sys);
  if (sv->map_spmv.bytes < sizeof(int) * (ts + tv)) ALLOC(c, sv->map_spmv, 2 * want_map);
  if (sv->status_dev.bytes < sizeof(int) * kStatusInts * n) ALLOC(c, sv->status_dev, 2 * kStatusInts * sizeof(int) * std::max(n, 64));
  HIPCHK(c, hipMemcpyAsync(sv->sys_dev.p, sv->h_sys, sizeof(PcgSystem) * n, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(sv->map_spmv.p, sv->h_map, sizeof(int) * (ts + tv), hipMemcpyHostToDevice, c->stream));
  *nwg_spmv = ts;
  *nwg_vec = tv;
  return BF_OK;
}

// Copy out the result of a finished system and release its slot.
void retire(bf_server* sv, int si, const int* stat) {
  bf_context* c = sv->batch_ctx;
  Slot& sl = sv->slots[si];
  Request* r = sl.req;
  bf_problem* pb = sl.pb;
  hipStream_t s = c->stream;
  bf_status st = BF_OK;
  std::string msg;
  const int n = pb->n_c;
  pb->ctx = c;
  launch_pcg_finish(sl.S, pb->Linv.as<double>(), pb->pout.as<double>(), pb->viol_part.as<double>(),
                    div_up(n, kBlock) > 0 ? div_up(n, kBlock) : 1, s);
  r->p.resize(3LL * pb->N);
  int nnzb = 0;
  hipError_t e = hipMemcpyAsync(r->p.data(), pb->pout.p, 24LL * pb->N, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(pb->host_sc, sl.S.sc, sizeof(PcgScalars), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&nnzb, pb->row_ptr.as<int>() + pb->N, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    st = BF_ERR_HIP;
    msg = hipGetErrorString(e);
  } else {
    const PcgScalars& h = *pb->host_sc;
    bf_step_stats& o = r->stats;
    o = bf_step_stats{};
    o.pcg_iters = h.iter;
    o.rel_residual = h.bb > 0.0 ? std::sqrt(h.rr_true / h.bb) : 0.0;
    o.newton_inf_over_h = h.stat_pinf / pb->dt;
    o.max_violation = h.stat_viol;
    o.nnzb = nnzb;
    o.ms_assemble = r->ms_setup;
    if (stat[1] || (stat[3] & (FLAG_NOT_SPD | FLAG_BREAKDOWN))) {
      st = BF_ERR_NOT_SPD;
      msg = "matrix not SPD (PCG breakdown)";
    } else if (stat[0] == 2) {
      st = BF_WARN_PCG_MAXITER;
      msg = "PCG reached max_iter";
    }
  }
  pb->stepped = true;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    (void)bf_admission_release(sv->adm, si, r->footprint);
    sl.req = nullptr;
  }
  r->stats.ms_pcg = (now_s() - r->t_admit) * 1e3 - r->ms_setup;
  finish_request(sv, r, st, msg);
  sv->cv.notify_all();
}

void batch_loop(bf_server* sv) {
  bf_context* c = sv->batch_ctx;
  (void)hipSetDevice(c->device);
  hipStream_t s = c->stream;
  bool changed = false;
  int nwg_spmv = 0, nwg_vec = 0;
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      while (!sv->stop && sv->ready.empty() && sv->active.empty()) sv->cv.wait(lk);
      if (sv->stop) return;
      while (!sv->ready.empty()) {
        sv->active.push_back(sv->ready.front());
        sv->ready.pop_front();
        changed = true;
      }
    }
    if (changed) {
      if (upload_table(sv, &nwg_spmv, &nwg_vec) != BF_OK) {
        // cannot run the batch: fail every active request
        for (int si : sv->active) {
          Request* r = sv->slots[si].req;
          {
            std::lock_guard<std::mutex> lk(sv->mu);
            (void)bf_admission_release(sv->adm, si, r->footprint);
            sv->slots[si].req = nullptr;
          }
          finish_request(sv, r, BF_ERR_HIP, c->err);
        }
        sv->active.clear();
        sv->cv.notify_all();
        continue;
      }
      changed = false;
    }
    const PcgSystem* sys = sv->sys_dev.as<PcgSystem>();
    const int* map = sv->map_spmv.as<int>();
    for (int k = 0; k < sv->iters_per_round; ++k)
      launch_pcg_iteration_batched(sys, map, nwg_spmv, map + nwg_spmv, nwg_vec, false, s);
    const int n = (int)sv->active.size();
    hipLaunchKernelGGL(k_gather_status, dim3(div_up(n, kBlock)), dim3(kBlock), 0, s, sys, n,
                       sv->status_dev.as<int>());
    hipError_t e = hipMemcpyAsync(sv->h_status, sv->status_dev.p, sizeof(int) * kStatusInts * n,
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      c->err = hipGetErrorString(e);
      for (int si : sv->active) {
        Request* r = sv->slots[si].req;
        {
          std::lock_guard<std::mutex> lk(sv->mu);
          (void)bf_admission_release(sv->adm, si, r->footprint);
          sv->slots[si].req = nullptr;
        }
        finish_request(sv, r, BF_ERR_HIP, c->err);
      }
      sv->active.clear();
      sv->cv.notify_all();
      continue;
    }
    std::vector<int> keep;
    for (int k = 0; k < n; ++k) {
      const int* st = sv->h_status + kStatusInts * k;
      if (st[0] == 4 && !st[1]) {   // residual replacement requested: the system stays in the batch
        bf_problem* pb = sv->slots[sv->active[k]].pb;
        launch_pcg_replace(sv->slots[sv->active[k]].S, pb->bhat.as<float>(), pb->rd.as<double>(),
                           pb->rpart.as<double>(), s);
        keep.push_back(sv->active[k]);
      } else if (st[0] || st[1]) {
        retire(sv, sv->active[k], st);
        changed = true;
      } else {
        keep.push_back(sv->active[k]);
      }
    }
    sv->active.swap(keep);
  }
}

template <class T>
void copy_in(std::vector<T>& v, const T* p, long long n) {
  if (p && n > 0) v.assign(p, p + n); else v.clear();
}

}  // namespace

extern "C" {

double bf_clock_now(void) { return now_s(); }

bf_status bf_server_create(int32_t device, const bf_server_opts* o, bf_server** out) {
  if (!out || !o) return BF_ERR_INVALID_ARG;
  *out = nullptr;
  if (o->max_active < 1 || o->iters_per_round < 1 || o->hbm_budget == 0 || o->admit_threads < 0 ||
      o->admit_threads > 64)
    return BF_ERR_INVALID_ARG;
  bf_server* sv = new (std::nothrow) bf_server();
  if (!sv) return BF_ERR_OOM;
  // three admission streams and the batch stream: within the four hardware
  // queues a process gets by default, so the batch never shares one
  const int nadmit = o->admit_threads > 0 ? o->admit_threads : 3;
  bf_status st = bf_context_create(device, nullptr, &sv->batch_ctx);
  for (int i = 0; i < nadmit && st == BF_OK; ++i) {
    bf_context* c = nullptr;
    st = bf_context_create(device, nullptr, &c);
    if (st == BF_OK) sv->admit_ctx.push_back(c);
  }
  if (st != BF_OK) {
    bf_server_destroy(sv);
    return st;
  }
  st = bf_admission_create(o->hbm_budget, o->max_active, &sv->adm);
  if (st != BF_OK) {
    bf_server_destroy(sv);
    return st;
  }
  sv->max_active = o->max_active;
  sv->iters_per_round = o->iters_per_round;
  sv->slots.resize(o->max_active);
  for (int i = 0; i < nadmit; ++i) sv->admit_threads.emplace_back(admission_loop, sv, i);
  sv->batch_thread = std::thread(batch_loop, sv);
  *out = sv;
  return BF_OK;
}

bf_status bf_server_submit(bf_server* sv, int64_t req_id, const bf_mesh_desc* m, const double* x,
                           const double* x_hat, const double* x_tilde, double dt, const bf_constraint_desc* cd,
                           const bf_solve_opts* opts) {
  if (!sv || !m || !cd || !opts) return BF_ERR_INVALID_ARG;
  // the request's host arrays, checked here as bf_problem_create, bf_set_state,
  // bf_set_constraints and bf_newton_step check them (the FP32 mode only)
  bf_status chk = bf_check_mesh(m, nullptr, 0);
  if (chk == BF_OK) chk = bf_check_state(m->n_nodes, x, x_hat, x_tilde, dt, nullptr, 0);
  if (chk == BF_OK) chk = bf_check_constraints(m->n_nodes, cd, nullptr, 0);
  if (chk == BF_OK) chk = bf_check_solve_opts(opts, nullptr, 0);
  if (chk != BF_OK) return chk;
  if (opts->precision != BF_PREC_FP32) return BF_ERR_INVALID_ARG;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->done.count(req_id)) return BF_ERR_INVALID_ARG;
    for (const Request* q : sv->pending)
      if (q->id == req_id) return BF_ERR_INVALID_ARG;
  }
  Request* r = new (std::nothrow) Request();
  if (!r) return BF_ERR_OOM;
  r->t_submit = now_s();
  r->id = req_id;
  r->N = m->n_nodes;
  r->T = m->n_tets;
  r->n_pt = cd->n_pt;
  r->n_ee = cd->n_ee;
  const long long N = m->n_nodes, T = m->n_tets, nc = (long long)cd->n_pt + cd->n_ee;
  copy_in(r->tets, m->tets, 4 * T);
  copy_in(r->rest, m->rest, 3 * N);
  copy_in(r->E, m->E, T);
  copy_in(r->nu, m->nu, T);
  copy_in(r->rho, m->rho, T);
  copy_in(r->fixed, m->fixed, N);
  copy_in(r->material, m->material, T);
  copy_in(r->x, x, 3 * N);
  copy_in(r->xh, x_hat, 3 * N);
  copy_in(r->xt, x_tilde, 3 * N);
  copy_in(r->pt, cd->pt, 4LL * cd->n_pt);
  copy_in(r->ee, cd->ee, 4LL * cd->n_ee);
  copy_in(r->lam, cd->lambda, nc);
  copy_in(r->gam, cd->gamma, nc);
  r->dt = dt;
  r->kappa = cd->kappa;
  r->delta = cd->delta;
  r->opts = *opts;
  if (bf_footprint_bytes(m->n_nodes, m->n_tets, (int32_t)nc, &r->footprint) != BF_OK) {
    delete r;
    return BF_ERR_INVALID_ARG;
  }
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    const bf_status st = bf_admission_push(sv->adm, req_id, r->footprint);
    if (st != BF_OK) {
      delete r;
      return st;
    }
    sv->pending.push_back(r);
  }
  sv->cv.notify_all();
  return BF_OK;
}

bf_status bf_server_poll(bf_server* sv, int64_t* done_ids, int32_t cap, int32_t* n_done) {
  if (!sv || !n_done || (cap > 0 && !done_ids) || cap < 0) return BF_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(sv->mu);
  const int n = std::min<int>(cap, (int)sv->done_unreported.size());
  for (int i = 0; i < n; ++i) done_ids[i] = sv->done_unreported[i];
  sv->done_unreported.erase(sv->done_unreported.begin(), sv->done_unreported.begin() + n);
  *n_done = n;
  return BF_OK;
}

bf_status bf_server_result(bf_server* sv, int64_t req_id, double* p_out, bf_step_stats* stats,
                           bf_request_times* times, int32_t* req_status) {
  if (!sv) return BF_ERR_INVALID_ARG;
  Request* r = nullptr;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->done.find(req_id);
    if (it == sv->done.end()) return BF_ERR_STATE;
    r = it->second;
    sv->done.erase(it);
  }
  if (p_out && !r->p.empty()) std::copy(r->p.begin(), r->p.end(), p_out);
  if (stats) *stats = r->stats;
  if (times) {
    times->t_submit = r->t_submit;
    times->t_admit = r->t_admit;
    times->t_done = r->t_done;
  }
  if (req_status) *req_status = r->status;
  delete r;
  return BF_OK;
}

bf_status bf_server_stats(bf_server* sv, int32_t* n_pending, int32_t* n_active, size_t* used_bytes) {
  if (!sv) return BF_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(sv->mu);
  if (n_pending) *n_pending = bf_admission_waiting(sv->adm);
  if (n_active) *n_active = bf_admission_active(sv->adm);
  if (used_bytes) *used_bytes = (size_t)bf_admission_used(sv->adm);
  return BF_OK;
}

void bf_server_destroy(bf_server* sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->cv.notify_all();
  for (std::thread& t : sv->admit_threads)
    if (t.joinable()) t.join();
  if (sv->batch_thread.joinable()) sv->batch_thread.join();
  if (sv->batch_ctx) (void)hipStreamSynchronize(sv->batch_ctx->stream);
  for (bf_context* c : sv->admit_ctx) (void)hipStreamSynchronize(c->stream);
  for (Slot& sl : sv->slots)
    if (sl.pb) bf_problem_destroy(sl.pb);
  for (Request* r : sv->pending) delete r;
  bf_admission_destroy(sv->adm);
  for (auto& kv : sv->done) delete kv.second;
  for (auto& sl : sv->slots) delete sl.req;
  sv->sys_dev.release();
  sv->map_spmv.release();
  sv->map_vec.release();
  sv->status_dev.release();
  if (sv->h_sys) (void)hipHostFree(sv->h_sys);
  if (sv->h_map) (void)hipHostFree(sv->h_map);
  if (sv->h_status) (void)hipHostFree(sv->h_status);
  for (bf_context* c : sv->admit_ctx) bf_context_destroy(c);
  bf_context_destroy(sv->batch_ctx);
  delete sv;
}

}  // extern "C"
