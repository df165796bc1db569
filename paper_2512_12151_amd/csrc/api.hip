// Host side of libbfal: the C-ABI declared in include/bfal.h.  Validates
// arguments, owns device memory, and enqueues the per-mesh setup and the
// per-Newton-step pipeline on the context's stream:
//   linearize constraints -> merged BSR pattern -> element kernel -> row
//   assembly (G, H, DBC, block-Jacobi factors) -> scaled off-diagonal blocks
//   -> PCG (device-side convergence flag, polled every poll_every iterations)
//   -> p = L^{-T} p_hat and FP64 stats.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "problem.h"

using namespace bfal;

namespace {

// Scratch of bf_energy_noalloc: the energy's per-workgroup partials, their
// sum and the inversion flag, in a file-scope device array (each GPU holds its
// own copy).  Host code never passes the array's name to a kernel: its device
// address is looked up once per device when a context is created and kept in
// g_scratch (the name is only a host-side stand-in).
constexpr size_t kScratchBytes = size_t(1) << 20;
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// With `device` current: the device address of `scratch` on it (looked up on
// the first call per device).
hipError_t scratch_lookup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch[device]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e == hipSuccess) g_scratch[device] = ptr;
  return e;
}

void* scratch_of(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return (device >= 0 && device < kMaxDevices) ? g_scratch[device] : nullptr;
}

}  // namespace

namespace bfal {

bf_status problem_init(bf_context* c, bf_problem* pb, const bf_mesh_desc* m, int32_t mem) {
  if (mem != BF_MEM_HOST && mem != BF_MEM_DEVICE) return fail(c, BF_ERR_INVALID_ARG, "mem must be BF_MEM_HOST or BF_MEM_DEVICE");
  {
    char msg[160];
    bf_status st = BF_OK;
    if (mem == BF_MEM_HOST) {
      st = bf_check_mesh(m, msg, sizeof msg);
    } else if (!m || !m->tets || !m->rest || !m->E || !m->nu || !m->rho) {
      st = BF_ERR_INVALID_ARG;
      std::snprintf(msg, sizeof msg, "mesh descriptor or one of its arrays is NULL");
    } else if (m->n_nodes <= 0 || m->n_tets <= 0) {
      st = BF_ERR_INVALID_ARG;
      std::snprintf(msg, sizeof msg, "n_nodes and n_tets must be positive");
    } else if ((long long)m->n_tets * 10 >= (1LL << 31) || (long long)m->n_nodes * 3 >= (1LL << 31)) {
      st = BF_ERR_INVALID_ARG;
      std::snprintf(msg, sizeof msg, "mesh too large for 32-bit slot indices");
    }
    if (st != BF_OK) return fail(c, st, msg);
  }
  const int N = m->n_nodes, T = m->n_tets;
  HIPCHK(c, hipSetDevice(c->device));
  pb->ctx = c;
  pb->N = N;
  pb->T = T;
  pb->has_state = false;
  pb->stepped = false;
  pb->cap_nnzb = 0;
  hipStream_t s = c->stream;
  ALLOC(c, pb->tets, 16LL * T);
  ALLOC(c, pb->rest, 24LL * N);
  ALLOC(c, pb->E, 8LL * T);
  ALLOC(c, pb->nu, 8LL * T);
  ALLOC(c, pb->rho, 8LL * T);
  ALLOC(c, pb->fixed, N);
  ALLOC(c, pb->Dminv9, 72LL * T);   // FP64 [9][T]
  ALLOC(c, pb->vol, 4LL * T);
  ALLOC(c, pb->mu, 4LL * T);
  ALLOC(c, pb->lam, 4LL * T);
  ALLOC(c, pb->mass, 8LL * N);
  ALLOC(c, pb->flags, 64);
  HIPCHK(c, hipMemcpyAsync(pb->tets.p, m->tets, 16LL * T, kind_in(mem), s));
  HIPCHK(c, hipMemcpyAsync(pb->rest.p, m->rest, 24LL * N, kind_in(mem), s));
  HIPCHK(c, hipMemcpyAsync(pb->E.p, m->E, 8LL * T, kind_in(mem), s));
  HIPCHK(c, hipMemcpyAsync(pb->nu.p, m->nu, 8LL * T, kind_in(mem), s));
  HIPCHK(c, hipMemcpyAsync(pb->rho.p, m->rho, 8LL * T, kind_in(mem), s));
  pb->has_mat = m->material != nullptr;
  pb->n_f = 0;   // a reused problem object starts without a friction set
  if (pb->has_mat) {
    ALLOC(c, pb->mat, 4LL * T);
    HIPCHK(c, hipMemcpyAsync(pb->mat.p, m->material, 4LL * T, kind_in(mem), s));
  }
  if (m->fixed) {
    HIPCHK(c, hipMemcpyAsync(pb->fixed.p, m->fixed, N, kind_in(mem), s));
  } else {
    std::vector<uint8_t> z(N, 0);
    HIPCHK(c, hipMemcpyAsync(pb->fixed.p, z.data(), N, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipStreamSynchronize(s));
  }
  int* flags = pb->flags.as<int>();
  fill_int(flags, 0, 16, s);
  const int4* tets = pb->tets.as<int4>();
  launch_check_tets(tets, T, N, flags, s);
  int hflags = 0;
  bf_status r0 = read_flags(pb, &hflags);
  if (r0 != BF_OK) return r0;
  if (hflags) return flags_to_status(c, hflags);
  launch_rest_geometry(tets, pb->rest.as<double>(), pb->E.as<double>(), pb->nu.as<double>(), pb->rho.as<double>(), T,
                       pb->Dminv9.as<double>(), pb->vol.as<float>(), pb->mu.as<float>(), pb->lam.as<float>(), flags, s);
  // static elastic pattern: pair keys bucketed by row, sorted and unique per row
  const long long npairs = 6LL * T;
  const long long nslots_tmp = (long long)N + 1;
  ALLOC(c, pb->scratch_int, 4LL * (3 * nslots_tmp + npairs + 16));
  int* cnt = pb->scratch_int.as<int>();
  int* kptr = cnt + nslots_tmp;
  int* cursor = kptr + nslots_tmp;
  int* keys = cursor + nslots_tmp;
  ALLOC(c, pb->scan_tmp, 4LL * scan_tmp_ints(10LL * T + N + 16));
  int* tmp = pb->scan_tmp.as<int>();
  fill_int(cnt, 0, N, s);
  launch_elastic_pair_count(tets, T, cnt, s);
  scan_exclusive(cnt, kptr, N, kptr + N, tmp, s);
  fill_int(cursor, 0, N, s);
  launch_elastic_pair_fill(tets, T, kptr, cursor, keys, s);
  ALLOC(c, pb->erow_ptr, 4LL * (N + 1));
  int* ucount = cnt;  // reuse
  launch_row_unique(keys, kptr, N, ucount, s);
  int* erow = pb->erow_ptr.as<int>();
  scan_exclusive(ucount, erow, N, erow + N, tmp, s);
  int nnzb_e = 0;
  HIPCHK(c, hipMemcpyAsync(&nnzb_e, erow + N, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  pb->nnzb_e = nnzb_e;
  ALLOC(c, pb->ecol, 4LL * nnzb_e);
  launch_row_write(keys, kptr, N, erow, pb->ecol.as<int>(), s);
  // (tet, pair) -> elastic slot, and each slot's contributions in (tet, pair) order
  ALLOC(c, pb->emap, 40LL * T);
  launch_emap(tets, T, erow, pb->ecol.as<int>(), pb->emap.as<int>(), s);
  ALLOC(c, pb->ecptr, 4LL * (nnzb_e + 1));
  ALLOC(c, pb->elist, 40LL * T);
  ALLOC(c, pb->epos, 40LL * T);
  // nnzb_e <= N + 6T, so the scratch buffer already holds nnzb_e counters
  int* scnt = pb->scratch_int.as<int>();
  int* ecptr = pb->ecptr.as<int>();
  fill_int(scnt, 0, nnzb_e, s);
  launch_slot_count(pb->emap.as<int>(), 10LL * T, scnt, s);
  scan_exclusive(scnt, ecptr, nnzb_e, ecptr + nnzb_e, tmp, s);
  fill_int(scnt, 0, nnzb_e, s);
  launch_slot_fill(pb->emap.as<int>(), 10LL * T, ecptr, scnt, pb->elist.as<int>(), s);
  sort_segments(pb->elist.as<int>(), ecptr, nnzb_e, s);
  launch_inverse_positions(pb->elist.as<int>(), 10LL * T, pb->epos.as<int>(), s);
  launch_mass(ecptr, pb->elist.as<int>(), erow, pb->vol.as<float>(), pb->rho.as<double>(), N, pb->mass.as<double>(), s);
  ALLOC(c, pb->staging, 720LL * T);   // FP64: ten 3x3 blocks (the diagonal ones with the gradient) per tet
  r0 = read_flags(pb, &hflags);
  if (r0 != BF_OK) return r0;
  if (hflags) return flags_to_status(c, hflags);
  for (auto& e : pb->ev)
    if (!e) HIPCHK(c, hipEventCreate(&e));
  if (!pb->host_sc) HIPCHK(c, hipHostMalloc((void**)&pb->host_sc, sizeof(PcgScalars), hipHostMallocDefault));
  ALLOC(c, pb->scal, sizeof(PcgScalars));
  HIPCHK(c, hipMemsetAsync(pb->scal.p, 0, sizeof(PcgScalars), s));
  HIPCHK(c, hipStreamSynchronize(s));
  return BF_OK;
}

}  // namespace bfal

namespace bfal {

bf_status step_assemble(bf_problem* pb, bool bf16) {
  bf_context* c = pb->ctx;
  HIPCHK(c, hipSetDevice(c->device));
  hipStream_t s = c->stream;
  const int N = pb->N, T = pb->T, n = pb->n_c, nf = pb->n_f;
  int* flags = pb->flags.as<int>();
  int* tmp = pb->scan_tmp.as<int>();
  const int4* ids = pb->cids.as<int4>();
  const int4* pids = ids;   // the pattern's stencils
  int npat = n;
  fill_int(flags, 0, 16, s);
  HIPCHK(c, hipEventRecord(pb->ev[0], s));
  // (1) constraint linearization at x and AL factors at x_hat
  fill_int(reinterpret_cast<int*>(pb->viol_part.p), 0, 2, s);
  launch_contact_lin(ids, pb->n_pt, n, pb->x.as<double>(), pb->xh.as<double>(), pb->clam.as<double>(),
                     pb->cgam.as<double>(), pb->kappa, pb->delta, pb->cg.as<double>(), pb->ch.as<double>(),
                     pb->lin64.as<double>(), pb->viol_part.as<double>(), flags, s);
  HIPCHK(c, hipEventRecord(pb->ev[1], s));
  // (2) merged pattern: vertex -> constraint incidence, candidates, unique rows.
  // Its stencils: the constraints, then the friction contacts that match no
  // constraint (a matched contact adds its terms at its constraint's incidences)
  if (nf > 0) {
    const unsigned cap = friction_table_capacity(n);
    int* cfr = pb->cfr.as<int>();
    int* extra = pb->fextra.as<int>();
    int* pos = pb->fpos.as<int>();
    fill_int(pb->ftab.as<int>(), -1, cap, s);
    fill_int(cfr, -1, n + 1, s);
    launch_stencil_insert(ids, n, pb->ftab.as<int>(), cap - 1, s);
    launch_friction_match(pb->fids.as<int4>(), nf, ids, pb->ftab.as<int>(), cap - 1, cfr, extra, s);
    scan_exclusive(extra, pos, nf, pos + nf, tmp, s);
    int n_extra = 0;
    HIPCHK(c, hipMemcpyAsync(&n_extra, pos + nf, sizeof(int), hipMemcpyDeviceToHost, s));
    if (n) HIPCHK(c, hipMemcpyAsync(pb->pids.p, pb->cids.p, 16LL * n, hipMemcpyDeviceToDevice, s));
    launch_friction_extra(pb->fids.as<int4>(), nf, extra, pos, n, pb->pids.as<int4>(), pb->fext.as<int>(), s);
    HIPCHK(c, hipStreamSynchronize(s));
    pids = pb->pids.as<int4>();
    npat = n + n_extra;
  }
  int* vcnt = pb->vcnt.as<int>();
  int* vptr = pb->vptr.as<int>();
  fill_int(vcnt, 0, N, s);
  launch_vertex_incidence_count(pids, npat, vcnt, s);
  scan_exclusive(vcnt, vptr, N, vptr + N, tmp, s);
  fill_int(vcnt, 0, N, s);
  launch_vertex_incidence_fill(pids, npat, vptr, vcnt, pb->vinc.as<int>(), s);
  sort_segments(pb->vinc.as<int>(), vptr, N, s);
  int* cptr = pb->cptr.as<int>();
  launch_candidate_count(pb->erow_ptr.as<int>(), vptr, pb->vinc.as<int>(), pids, N, pb->ccount.as<int>(), s);
  scan_exclusive(pb->ccount.as<int>(), cptr, N, cptr + N, tmp, s);
  launch_candidate_fill(pb->erow_ptr.as<int>(), pb->ecol.as<int>(), vptr, pb->vinc.as<int>(), pids, N, cptr,
                        pb->cand.as<int>(), pb->ucount.as<int>(), s);
  int* row_ptr = pb->row_ptr.as<int>();
  scan_exclusive(pb->ucount.as<int>(), row_ptr, N, row_ptr + N, tmp, s);
  launch_merged_write(pb->cand.as<int>(), cptr, row_ptr, pb->erow_ptr.as<int>(), pb->ecol.as<int>(), N,
                      pb->col.as<int>(), pb->eslot.as<int>(), s);
  // slots of every stencil's ten vertex pairs in the merged pattern, for the row assembly
  ALLOC(c, pb->cslot, 40LL * npat + 16);
  launch_cmap(pids, npat, row_ptr, pb->col.as<int>(), pb->cslot.as<int>(), s);
  HIPCHK(c, hipEventRecord(pb->ev[2], s));
  // (3) assembly (friction terms at x_hat first)
  launch_friction_terms(pb->fids.as<int4>(), nf, pb->xh.as<double>(), pb->fx0.as<double>(), pb->f64.as<double>(),
                        pb->fric_e, pb->fgk.as<double>(), s);
  const double h2 = pb->dt * pb->dt;
  launch_elastic(pb->tets.as<int4>(), T, pb->rest.as<double>(), pb->xh.as<double>(), pb->Dminv9.as<double>(),
                 pb->vol.as<float>(), pb->mu.as<float>(), pb->lam.as<float>(), h2, pb->epos.as<int>(),
                 pb->staging.as<double>(), pb->has_mat ? pb->mat.as<int>() : nullptr, flags, s);
  launch_assemble_rows(N, pb->cap_nnzb, row_ptr, pb->col.as<int>(), pb->eslot.as<int>(), pb->erow_ptr.as<int>(),
                       pb->ecol.as<int>(), pb->ecptr.as<int>(), pb->staging.as<double>(), vptr, pb->vinc.as<int>(),
                       pids, pb->cslot.as<int>(), n, pb->lin64.as<double>(),
                       pb->cg.as<double>(), pb->ch.as<double>(), nf, pb->fgk.as<double>(), pb->cfr.as<int>(),
                       pb->fext.as<int>(), pb->mass.as<double>(), pb->xh.as<double>(), pb->xt.as<double>(),
                       pb->fixed.as<uint8_t>(), pb->vals.as<double>(), pb->grad.as<float>(), pb->Lf.as<float>(),
                       pb->Linv.as<double>(), pb->bhat.as<float>(), pb->bb_part.as<double>(), flags, s);
  // sliced storage of the scaled matrix: per column the source rows of its
  // upper blocks, slot counts per slice, then the slots themselves
  int* lcnt = pb->lcnt.as<int>();
  int* lptr = pb->lptr.as<int>();
  fill_int(lcnt, 0, N, s);
  launch_lower_count(N, row_ptr, pb->col.as<int>(), lcnt, s);
  scan_exclusive(lcnt, lptr, N, lptr + N, tmp, s);
  fill_int(lcnt, 0, N, s);
  launch_lower_fill(N, row_ptr, pb->col.as<int>(), lptr, lcnt, pb->lsrc.as<int>(), s);
  sort_segments(pb->lsrc.as<int>(), lptr, N, s);
  const int nslices = div_up(N, kSlice);
  int* sbu = pb->sbu.as<int>();
  int* sbl = pb->sbl.as<int>();
  int* wmax = pb->scratch_int.as<int>();   // free after the per-mesh setup
  fill_int(wmax, 0, 2, s);
  launch_slice_widths(N, nslices, row_ptr, lptr, sbu, sbl, wmax, s);
  scan_exclusive(sbu, sbu, nslices, sbu + nslices, tmp, s);
  scan_exclusive(sbl, sbl, nslices, sbl + nslices, tmp, s);
  // the slot offsets come to the host for the SpMV's slice plan (bf_slice_plan)
  int tot[4] = {0, 0, 0, 0};
  pb->h_sbu.resize(nslices + 1);
  pb->h_sbl.resize(nslices + 1);
  HIPCHK(c, hipMemcpyAsync(pb->h_sbu.data(), sbu, 4LL * (nslices + 1), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipMemcpyAsync(pb->h_sbl.data(), sbl, 4LL * (nslices + 1), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipMemcpyAsync(&tot[2], wmax, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  tot[0] = pb->h_sbu[nslices];
  tot[1] = pb->h_sbl[nslices];
  pb->nslot_u = tot[0];
  pb->nslot_l = tot[1];
  const int nparts = kSpmvWaves * pcg_spmv_groups(N, c->num_cu);
  pb->h_wptr.resize(nparts + 1);
  pb->h_wsl.resize(nslices);
  if (bf_slice_plan(nslices, pb->h_sbu.data(), pb->h_sbl.data(), kPairs, nparts, pb->h_wptr.data(),
                    pb->h_wsl.data()) != BF_OK)
    return fail(c, BF_ERR_INVALID_ARG, "the slice plan rejected the slot offsets");
  ALLOC(c, pb->wplan_ptr, 4LL * (nparts + 1));
  ALLOC(c, pb->wplan_sl, 4LL * nslices);
  HIPCHK(c, hipMemcpyAsync(pb->wplan_ptr.p, pb->h_wptr.data(), 4LL * (nparts + 1), hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(pb->wplan_sl.p, pb->h_wsl.data(), 4LL * nslices, hipMemcpyHostToDevice, s));
  // slot arrays with the zero block (upper) and the SpMV's read-ahead padding
  const long long nu_alloc = tot[0] + slot_padding(tot[3]);
  const long long nl_alloc = tot[1] + slot_padding(tot[2]);
  ALLOC(c, pb->sblk, 36LL * nu_alloc);
  if (bf16) ALLOC(c, pb->sblk16, 20LL * nu_alloc);
  ALLOC(c, pb->scol, 4LL * nu_alloc);
  ALLOC(c, pb->sent, 8LL * nl_alloc);
  HIPCHK(c, hipMemsetAsync(pb->sblk.as<char>() + 36LL * tot[0], 0, 36LL * (nu_alloc - tot[0]), s));
  if (bf16) HIPCHK(c, hipMemsetAsync(pb->sblk16.as<char>() + 20LL * tot[0], 0, 20LL * (nu_alloc - tot[0]), s));
  HIPCHK(c, hipMemsetAsync(pb->scol.as<char>() + 4LL * tot[0], 0, 4LL * (nu_alloc - tot[0]), s));
  HIPCHK(c, hipMemsetAsync(pb->sent.as<char>() + 8LL * tot[1], 0, 8LL * (nl_alloc - tot[1]), s));
  launch_sell_fill(N, nslices, row_ptr, pb->col.as<int>(), pb->vals.as<double>(), pb->Linv.as<double>(), lptr,
                   pb->lsrc.as<int>(), sbu, sbl, pb->sblk.as<float>(), bf16 ? pb->sblk16.as<uint32_t>() : nullptr,
                   pb->scol.as<int>(),
                   pb->sent.as<int2>(), s);
  return BF_OK;
}

}  // namespace bfal

extern "C" {

bf_status bf_context_create(int32_t device, void* hip_stream, bf_context** out) {
  if (!out) return BF_ERR_INVALID_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return BF_ERR_INVALID_ARG;
  bf_context* c = new (std::nothrow) bf_context();
  if (!c) return BF_ERR_OOM;
  c->device = device;
  if (hipSetDevice(device) != hipSuccess) { delete c; return BF_ERR_HIP; }
  if (scratch_lookup(device) != hipSuccess) { delete c; return BF_ERR_HIP; }
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && ncu > 0)
    c->num_cu = ncu;
  if (hip_stream) {
    c->stream = static_cast<hipStream_t>(hip_stream);
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) { delete c; return BF_ERR_HIP; }
    c->own_stream = true;
  }
  *out = c;
  return BF_OK;
}

void bf_context_destroy(bf_context* c) {
  if (!c) return;
  if (c->own_stream && c->stream) {
    (void)hipStreamSynchronize(c->stream);
    (void)hipStreamDestroy(c->stream);
  }
  delete c;
}

const char* bf_last_error(const bf_context* c) { return c ? c->err.c_str() : "null context"; }

bf_status bf_footprint_bytes(int32_t n_nodes, int32_t n_tets, int32_t n_constraints, size_t* out) {
  if (!out || n_nodes <= 0 || n_tets <= 0 || n_constraints < 0) return BF_ERR_INVALID_ARG;
  const size_t N = n_nodes, T = n_tets, C = n_constraints;
  const size_t nnzb_e = N + 6 * T;                 // upper bound on the static pattern
  const size_t cap = nnzb_e + 6 * C;
  size_t b = 0;
  b += T * (16 + 3 * 8 + 72 + 12 + 40 * 3 + 720);  // tets, E/nu/rho, Dm^-1, vol/mu/lam, emap/epos/elist, FP64 staging
  b += nnzb_e * (4 + 4) + N * (4 * 3 + 24 + 8 + 1);
  b += N * 24 * 3;                                 // x, x_hat, x_tilde
  b += C * (16 + 16 + 64 + 16 + 40);               // ids, lambda/gamma, FP64 linearization, AL factors, pair slots
  b += N * 4 * 8 + C * 16 + cap * 4 * 2;           // incidence, candidates, pattern
  b += cap * (72 + 36 + 4 + 4 + 8 + 4);            // FP64 blocks, FP32 scaled blocks, ucol, eslot, transpose index, lsrc
  b += N * (12 * (4 + kPRing) + 24 + 24 + 48 + 24);   // grad, bhat, r, q, the direction ring, x, L, L^-1, p out
  b += 1 << 20;                                    // partials, scalars, scan scratch, the SpMV slice plan
  b += 4 * (N / 64 + 1);
  *out = b;
  return BF_OK;
}

bf_status bf_problem_create(bf_context* c, const bf_mesh_desc* m, int32_t mem, bf_problem** out) {
  if (!c) return BF_ERR_INVALID_ARG;
  if (!out) return fail(c, BF_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  bf_problem* pb = new (std::nothrow) bf_problem();
  if (!pb) return fail(c, BF_ERR_OOM, "host allocation failed");
  pb->ctx = c;
  const bf_status st = problem_init(c, pb, m, mem);
  if (st != BF_OK) {
    bf_problem_destroy(pb);
    return st;
  }
  *out = pb;
  c->err.clear();
  return BF_OK;
}

void bf_problem_destroy(bf_problem* pb) {
  if (!pb) return;
  if (pb->ctx) (void)hipStreamSynchronize(pb->ctx->stream);
  DevBuf* bufs[] = {&pb->tets, &pb->rest, &pb->E, &pb->nu, &pb->rho, &pb->fixed, &pb->Dminv9, &pb->vol, &pb->mu,
                    &pb->lam, &pb->mass, &pb->erow_ptr, &pb->ecol, &pb->emap, &pb->ecptr, &pb->elist, &pb->epos,
                    &pb->staging, &pb->x, &pb->xh, &pb->xt, &pb->cids, &pb->clam, &pb->cgam,
                    &pb->cg, &pb->ch, &pb->viol_part, &pb->vcnt, &pb->vptr, &pb->vinc, &pb->ccount, &pb->cptr,
                    &pb->cand, &pb->ucount, &pb->row_ptr, &pb->col, &pb->eslot, &pb->vals, &pb->grad, &pb->Lf,
                    &pb->Linv, &pb->bhat, &pb->bb_part, &pb->lcnt, &pb->lptr, &pb->lsrc, &pb->sbu, &pb->sbl,
                    &pb->wplan_ptr, &pb->wplan_sl,                    &pb->sblk, &pb->sblk16, &pb->scol, &pb->sent, &pb->xs, &pb->r, &pb->pring, &pb->q,
                    &pb->part, &pb->scal, &pb->pout, &pb->flags, &pb->scan_tmp, &pb->scratch_int,
                    &pb->xd, &pb->rd, &pb->zd, &pb->fcg, &pb->rpart, &pb->lin64, &pb->pdir, &pb->xtrial,
                    &pb->epart, &pb->stris, &pb->sedges, &pb->sverts, &pb->xq, &pb->tbox, &pb->tkey, &pb->tkey2,
                    &pb->tchild, &pb->tparent, &pb->tnode, &pb->tarrive, &pb->ebox, &pb->ekey, &pb->ekey2,
                    &pb->echild, &pb->eparent, &pb->enode, &pb->earrive, &pb->bpart, &pb->qcount, &pb->qpairs[0],
                    &pb->qpairs[1], &pb->qtoc[0], &pb->qtoc[1], &pb->pkey, &pb->pkey2, &pb->pidx, &pb->pidx2,
                    &pb->sort_tmp, &pb->ctmp, &pb->htable, &pb->tvmin, &pb->keepn[0], &pb->keepn[1], &pb->posn[0],
                    &pb->posn[1], &pb->keepc, &pb->posc, &pb->nids, &pb->nlam, &pb->ngam, &pb->mpart,
                    &pb->xstart, &pb->xprev, &pb->vout, &pb->mat, &pb->fids, &pb->f64, &pb->fx0, &pb->fgk,
                    &pb->pids, &pb->cslot, &pb->ftab, &pb->cfr, &pb->fextra, &pb->fpos, &pb->fext};
  for (DevBuf* b : bufs) b->release();
  for (auto& e : pb->ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : pb->tev) (void)hipEventDestroy(e);
  if (pb->host_sc) (void)hipHostFree(pb->host_sc);
  delete pb;
}

bf_status bf_set_state(bf_problem* pb, const double* x, const double* x_hat, const double* x_tilde, double dt,
                       int32_t mem) {
  if (!pb) return BF_ERR_INVALID_ARG;
  bf_context* c = pb->ctx;
  if (mem != BF_MEM_HOST && mem != BF_MEM_DEVICE) return fail(c, BF_ERR_INVALID_ARG, "bad mem kind");
  {
    char msg[160];
    bf_status st = BF_OK;
    if (mem == BF_MEM_HOST) {
      st = bf_check_state(pb->N, x, x_hat, x_tilde, dt, msg, sizeof msg);
    } else if (!x || !x_hat || !x_tilde) {
      st = BF_ERR_INVALID_ARG;
      std::snprintf(msg, sizeof msg, "state array is NULL");
    } else if (!(dt > 0.0) || !std::isfinite(dt)) {
      st = BF_ERR_INVALID_ARG;
      std::snprintf(msg, sizeof msg, "dt must be positive and finite");
    }
    if (st != BF_OK) return fail(c, st, msg);
  }
  const long long n3 = 3LL * pb->N;
  ALLOC(c, pb->x, 8 * n3);
  ALLOC(c, pb->xh, 8 * n3);
  ALLOC(c, pb->xt, 8 * n3);
  HIPCHK(c, hipMemcpyAsync(pb->x.p, x, 8 * n3, kind_in(mem), c->stream));
  HIPCHK(c, hipMemcpyAsync(pb->xh.p, x_hat, 8 * n3, kind_in(mem), c->stream));
  HIPCHK(c, hipMemcpyAsync(pb->xt.p, x_tilde, 8 * n3, kind_in(mem), c->stream));
  if (mem == BF_MEM_HOST) HIPCHK(c, hipStreamSynchronize(c->stream));
  pb->dt = dt;
  pb->has_state = true;
  c->err.clear();
  return BF_OK;
}

bf_status bf_set_constraints(bf_problem* pb, const bf_constraint_desc* cd, int32_t mem) {
  if (!pb) return BF_ERR_INVALID_ARG;
  bf_context* c = pb->ctx;
  if (mem != BF_MEM_HOST && mem != BF_MEM_DEVICE) return fail(c, BF_ERR_INVALID_ARG, "bad mem kind");
  const int N = pb->N;
  {
    // a device descriptor: its scalars and pointers here, its contents in k_check_constraints below
    char msg[160];
    bf_status st = BF_OK;
    if (mem == BF_MEM_HOST) {
      st = bf_check_constraints(N, cd, msg, sizeof msg);
    } else if (cd) {
      const long long n_all = (long long)cd->n_pt + cd->n_ee;
      const bf_constraint_desc scalars{0, 0, nullptr, nullptr, nullptr, nullptr, cd->kappa, cd->delta};
      st = BF_ERR_INVALID_ARG;
      if (cd->n_pt < 0 || cd->n_ee < 0)
        std::snprintf(msg, sizeof msg, "negative constraint count");
      else if (n_all * 10 >= (1LL << 31))
        std::snprintf(msg, sizeof msg, "too many constraints");
      else if ((cd->n_pt && !cd->pt) || (cd->n_ee && !cd->ee) || (n_all && !cd->lambda))
        std::snprintf(msg, sizeof msg, "constraint array is NULL");
      else
        st = bf_check_constraints(N, &scalars, msg, sizeof msg);
    } else {
      st = bf_check_constraints(N, cd, msg, sizeof msg);
    }
    if (st != BF_OK) return fail(c, st, msg);
  }
  const long long nc = (long long)cd->n_pt + cd->n_ee;
  hipStream_t s = c->stream;
  const int n = (int)nc;
  ALLOC(c, pb->cids, 16LL * n + 16);
  ALLOC(c, pb->clam, 8LL * n + 8);
  ALLOC(c, pb->cgam, 8LL * n + 8);
  if (cd->n_pt) HIPCHK(c, hipMemcpyAsync(pb->cids.p, cd->pt, 16LL * cd->n_pt, kind_in(mem), s));
  if (cd->n_ee)
    HIPCHK(c, hipMemcpyAsync(pb->cids.as<char>() + 16LL * cd->n_pt, cd->ee, 16LL * cd->n_ee, kind_in(mem), s));
  if (n) HIPCHK(c, hipMemcpyAsync(pb->clam.p, cd->lambda, 8LL * n, kind_in(mem), s));
  if (n && cd->gamma) {
    HIPCHK(c, hipMemcpyAsync(pb->cgam.p, cd->gamma, 8LL * n, kind_in(mem), s));
  } else if (n) {
    std::vector<double> ones(n, 1.0);
    HIPCHK(c, hipMemcpyAsync(pb->cgam.p, ones.data(), 8LL * n, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipStreamSynchronize(s));
  }
  if (mem == BF_MEM_DEVICE && n) {
    fill_int(pb->flags.as<int>(), 0, 16, s);
    launch_check_constraints(pb->cids.as<int4>(), n, N, pb->clam.as<double>(), pb->cgam.as<double>(),
                             pb->flags.as<int>(), s);
    int hflags = 0;
    bf_status r0 = read_flags(pb, &hflags);
    if (r0 != BF_OK) return r0;
    if (hflags) return flags_to_status(c, hflags);
  }
  HIPCHK(c, hipStreamSynchronize(s));
  pb->kappa = cd->kappa;
  pb->delta = cd->delta;
  return size_constraint_buffers(pb, cd->n_pt, cd->n_ee);
}

bf_status bf_set_friction(bf_problem* pb, double mu_f, double eps_v) {
  if (!pb) return BF_ERR_INVALID_ARG;
  bf_context* c = pb->ctx;
  if (!(mu_f >= 0.0) || !std::isfinite(mu_f)) return fail(c, BF_ERR_INVALID_ARG, "mu_f must be finite and >= 0");
  if (mu_f > 0.0 && (!(eps_v > 0.0) || !std::isfinite(eps_v)))
    return fail(c, BF_ERR_INVALID_ARG, "eps_v must be positive and finite");
  if (!pb->has_state) return fail(c, BF_ERR_STATE, "bf_set_friction needs the state (bf_set_state) first");
  if (pb->cap_nnzb == 0) return fail(c, BF_ERR_STATE, "bf_set_friction needs the constraints (bf_set_constraints) first");
  const int nf = mu_f > 0.0 ? pb->n_c : 0;
  if (nf == 0 && pb->n_f == 0) {   // no friction before or after: nothing to change
    c->err.clear();
    return BF_OK;
  }
  HIPCHK(c, hipSetDevice(c->device));
  hipStream_t s = c->stream;
  if (nf > 0) {
    ALLOC(c, pb->fids, 16LL * nf);
    ALLOC(c, pb->f64, 64LL * nf);
    ALLOC(c, pb->fgk, 104LL * nf);
    ALLOC(c, pb->fx0, 24LL * pb->N);
    HIPCHK(c, hipMemcpyAsync(pb->fids.p, pb->cids.p, 16LL * nf, hipMemcpyDeviceToDevice, s));
    HIPCHK(c, hipMemcpyAsync(pb->fx0.p, pb->x.p, 24LL * pb->N, hipMemcpyDeviceToDevice, s));
    launch_friction_capture(pb->fids.as<int4>(), pb->n_pt, nf, pb->x.as<double>(), pb->clam.as<double>(), pb->kappa,
                            pb->delta, mu_f, pb->f64.as<double>(), s);
    HIPCHK(c, hipGetLastError());
  }
  pb->n_f = nf;
  pb->fric_e = eps_v * pb->dt;
  return size_constraint_buffers(pb, pb->n_pt, pb->n_ee);
}

}  // extern "C"

namespace bfal {

bf_status size_constraint_buffers(bf_problem* pb, int n_pt, int n_ee) {
  bf_context* c = pb->ctx;
  hipStream_t s = c->stream;
  const int N = pb->N;
  const int n = n_pt + n_ee;
  pb->n_pt = n_pt;
  pb->n_ee = n_ee;
  pb->n_c = n;
  // size the per-step buffers for this constraint count (the pattern also
  // holds the stencils of the friction contacts)
  const long long np = (long long)n + pb->n_f;
  const long long cap = (long long)pb->nnzb_e + 6LL * np;
  const long long capc = (long long)pb->nnzb_e - N + 6LL * np + 16;
  ALLOC(c, pb->lin64, 64LL * n + 64);
  ALLOC(c, pb->cg, 8LL * n + 16);
  ALLOC(c, pb->ch, 8LL * n + 16);
  ALLOC(c, pb->viol_part, 8LL * (div_up(n, kBlock) + 1));
  ALLOC(c, pb->vcnt, 4LL * (N + 1));
  ALLOC(c, pb->vptr, 4LL * (N + 1));
  ALLOC(c, pb->vinc, 16LL * np + 16);
  if (pb->n_f > 0) {
    ALLOC(c, pb->pids, 16LL * np + 16);
    ALLOC(c, pb->ftab, 4LL * friction_table_capacity(n));
    ALLOC(c, pb->cfr, 4LL * (n + 1));
    ALLOC(c, pb->fextra, 4LL * (pb->n_f + 1));
    ALLOC(c, pb->fpos, 4LL * (pb->n_f + 1));
    ALLOC(c, pb->fext, 4LL * (pb->n_f + 1));
  }
  ALLOC(c, pb->ccount, 4LL * (N + 1));
  ALLOC(c, pb->cptr, 4LL * (N + 1));
  ALLOC(c, pb->cand, 4LL * capc);
  ALLOC(c, pb->ucount, 4LL * (N + 1));
  ALLOC(c, pb->row_ptr, 4LL * (N + 1));
  ALLOC(c, pb->col, 4LL * cap);
  ALLOC(c, pb->eslot, 4LL * cap);
  ALLOC(c, pb->vals, 72LL * cap);   // FP64 assembled blocks
  ALLOC(c, pb->lcnt, 4LL * (N + 1));
  ALLOC(c, pb->lptr, 4LL * (N + 1));
  ALLOC(c, pb->lsrc, 4LL * cap);
  const long long nsl = div_up(N, kSlice);
  ALLOC(c, pb->sbu, 4LL * (nsl + 1));
  ALLOC(c, pb->sbl, 4LL * (nsl + 1));
  // sliced storage: sized here for about 25 % padding, grown in the step if needed
  const long long slots0 = (cap - N) + (cap - N) / 4 + kSlice;
  ALLOC(c, pb->sblk, 36LL * (slots0 + 1));
  ALLOC(c, pb->scol, 4LL * slots0);
  ALLOC(c, pb->sent, 8LL * slots0);
  // solver vectors and the factor L are padded to a multiple of 4 nodes (float4
  // access); the pads are zeroed here and never written with nonzeros
  const long long N4 = (N + 3) & ~3LL;
  ALLOC(c, pb->grad, 12LL * N);
  ALLOC(c, pb->Lf, 24LL * N4);
  ALLOC(c, pb->Linv, 48LL * N4);   // FP64 L^{-1} per node (6 entries)
  ALLOC(c, pb->bhat, 12LL * N4);
  ALLOC(c, pb->bb_part, 8LL * (div_up(N, kBlock) + 1));
  ALLOC(c, pb->xs, 24LL * N4);   // FP64 solution
  ALLOC(c, pb->rd, 24LL * N4);   // FP64 residual (replacement, refinement)
  ALLOC(c, pb->rpart, 8LL * (kMaxSpmvParts + 8 + 6 * 256 + 8));
  ALLOC(c, pb->r, 12LL * N4);
  ALLOC(c, pb->pring, 12LL * N4 * kPRing);
  ALLOC(c, pb->q, 12LL * N4);
  for (DevBuf* b : {&pb->Lf, &pb->Linv, &pb->bhat, &pb->xs, &pb->rd, &pb->r, &pb->pring, &pb->q})
    HIPCHK(c, hipMemsetAsync(b->p, 0, b->bytes, s));
  HIPCHK(c, hipStreamSynchronize(s));
  ALLOC(c, pb->part, 8LL * kPartsPerSystem);
  ALLOC(c, pb->pout, 24LL * N);
  ALLOC(c, pb->scan_tmp, 4LL * scan_tmp_ints((long long)10 * pb->T + N + 6LL * np + 16));
  pb->cap_nnzb = cap;
  pb->cap_cand = capc;
  c->err.clear();
  return BF_OK;
}

}  // namespace bfal

extern "C" {

bf_status bf_newton_step(bf_problem* pb, const bf_solve_opts* o, double* p_out, int32_t mem, bf_step_stats* stats) {
  if (!pb) return BF_ERR_INVALID_ARG;
  bf_context* c = pb->ctx;
  if (!o || !p_out) return fail(c, BF_ERR_INVALID_ARG, "opts or p_out is NULL");
  if (!pb->has_state) return fail(c, BF_ERR_STATE, "bf_set_state must be called before bf_newton_step");
  if (pb->cap_nnzb == 0) return fail(c, BF_ERR_STATE, "bf_set_constraints must be called before bf_newton_step");
  {
    char msg[160];
    const bf_status st = bf_check_solve_opts(o, msg, sizeof msg);
    if (st != BF_OK) return fail(c, st, msg);
  }
  const bool bf16 = o->precision == BF_PREC_BF16_REFINE;
  if (mem != BF_MEM_HOST && mem != BF_MEM_DEVICE) return fail(c, BF_ERR_INVALID_ARG, "bad mem kind");
  HIPCHK(c, hipSetDevice(c->device));
  hipStream_t s = c->stream;
  const int N = pb->N, n = pb->n_c;
  int* flags = pb->flags.as<int>();
  int* row_ptr = pb->row_ptr.as<int>();
  {
    const bf_status r0 = step_assemble(pb, bf16);
    if (r0 != BF_OK) return r0;
  }
  PcgSystem S = system_of(pb);
  HIPCHK(c, hipEventRecord(pb->ev[3], s));
  // (4) PCG: one solve on the FP32 blocks, or iterative refinement around
  // solves on the BF16 copy
  const int poll = o->poll_every > 0 ? o->poll_every : 16;
  const int ntime = o->time_spmv > 0 ? (o->time_spmv < 4096 ? o->time_spmv : 4096) : 0;
  while ((int)pb->tev.size() < 2 * ntime) {
    hipEvent_t e;
    HIPCHK(c, hipEventCreate(&e));
    pb->tev.push_back(e);
  }
  int launched = 0, total_iters = 0, timed = 0, replacements = 0;
  bool assembly_checked = false;
  // Runs the solve set up on S to its device-side stop; the first poll also
  // checks the assembly's error flags.
  auto run_solve = [&](const PcgSystem& Sx, bool use_bf16) -> bf_status {
    int mine = 0;
    for (;;) {
      for (int k = 0; k < poll; ++k) {
        const bool t = launched + k < ntime;
        if (t)
          launch_pcg_iteration(Sx, use_bf16, s, pb->tev[2 * (launched + k)], pb->tev[2 * (launched + k) + 1]);
        else
          launch_pcg_iteration(Sx, use_bf16, s);
      }
      launched += poll;
      mine += poll;
      HIPCHK(c, hipMemcpyAsync(pb->host_sc, Sx.sc, sizeof(PcgScalars), hipMemcpyDeviceToHost, s));
      HIPCHK(c, hipStreamSynchronize(s));
      if (!assembly_checked) {
        int hf = 0;
        bf_status r0 = read_flags(pb, &hf);
        if (r0 != BF_OK) return r0;
        if (hf) return flags_to_status(c, hf);
        assembly_checked = true;
      }
      if (pb->host_sc->done == 4 && !pb->host_sc->brk) {   // residual replacement requested
        launch_pcg_replace(Sx, pb->bhat.as<float>(), pb->rd.as<double>(), pb->rpart.as<double>(), s);
        ++replacements;
        continue;
      }
      if (pb->host_sc->done || pb->host_sc->brk) break;
      if (mine > o->max_iter + poll + 64 * replacements) break;   // cannot happen: the device stops at max_iter
    }
    // every timed launch so far (early exits are filtered out below)
    timed = std::max(timed, std::min(ntime, launched));
    total_iters += pb->host_sc->iter;
    return BF_OK;
  };
  const int nviol = div_up(n, kBlock) > 0 ? div_up(n, kBlock) : 1;
  double sweep_res[16] = {0.0};
  int sweeps = 0;
  bool refine_capped = false;
  if (!bf16) {
    launch_pcg_init(S, pb->bhat.as<float>(), pb->bb_part.as<double>(), div_up(N, kBlock), o->tol, o->max_iter,
                    o->check_every, true, s);
    bf_status r0 = run_solve(S, false);
    if (r0 != BF_OK) return r0;
    launch_pcg_finish(S, pb->Linv.as<double>(), pb->pout.as<double>(), pb->viol_part.as<double>(), nviol, s);
  } else {
    // Flexible CG on the FP32-stored system in FP64 vectors (the refinement):
    // every sweep forms the true residual r = b_hat - H_hat x in FP64, solves
    // H_bf16 z = r by the two-kernel PCG on the BF16 blocks to the relative
    // tolerance tol (a BF16 breakdown ends that inner solve early: BF16
    // rounding can make the scaled matrix indefinite in its lowest modes),
    // makes z conjugate (in H_hat) to the last kFcgWindow directions, and
    // takes the exact step along it.  The outer Krylov recurrence on the FP32
    // operator recovers the modes the BF16 blocks cannot resolve.
    constexpr int kFcgWindow = 4;
    const long long n3 = 3LL * S.N4;
    ALLOC(c, pb->xd, 8 * n3);
    ALLOC(c, pb->rd, 8 * n3);
    ALLOC(c, pb->zd, 8 * n3);
    ALLOC(c, pb->fcg, 8 * n3 * 2 * kFcgWindow);
    ALLOC(c, pb->rpart, 8LL * (kMaxSpmvParts + 8 + 6 * 256 + 8));
    HIPCHK(c, hipMemsetAsync(pb->xd.p, 0, 8 * n3, s));
    HIPCHK(c, hipMemsetAsync(pb->rd.p, 0, 8 * n3, s));
    HIPCHK(c, hipMemsetAsync(pb->zd.p, 0, 8 * n3, s));
    HIPCHK(c, hipMemsetAsync(pb->fcg.p, 0, 8 * n3 * 2 * kFcgWindow, s));
    double* rpart = pb->rpart.as<double>();
    double* rsum = rpart + kMaxSpmvParts;        // [0] residual^2, [1] |b|^2
    double* dpart = rsum + 8;                    // partials of the dot products
    double* dots = dpart + 6 * 256;              // their sums
    double* xd = pb->xd.as<double>();
    double* rd = pb->rd.as<double>();
    double* zd = pb->zd.as<double>();
    auto Pv = [&](int j) { return pb->fcg.as<double>() + n3 * (2 * (j % kFcgWindow)); };
    auto Qv = [&](int j) { return pb->fcg.as<double>() + n3 * (2 * (j % kFcgWindow) + 1); };
    double pq_hist[kFcgWindow] = {0.0};
    launch_sum_to(pb->bb_part.as<double>(), div_up(N, kBlock), rsum + 1, s);
    PcgSystem S16 = S;
    S16.blk = pb->sblk16.p;
    const int max_sweeps = o->max_sweeps > 0 ? o->max_sweeps : 100;
    double bb = 0.0;
    for (int sw = 0;; ++sw) {
      launch_residual64(S, pb->bhat.as<float>(), xd, rd, rpart, rsum, s);
      double hs[2] = {0.0, 0.0};
      HIPCHK(c, hipMemcpyAsync(hs, rsum, sizeof(hs), hipMemcpyDeviceToHost, s));
      HIPCHK(c, hipStreamSynchronize(s));
      bb = hs[1];
      const double rel = bb > 0.0 ? std::sqrt(hs[0] / bb) : 0.0;
      if (sw < 16) sweep_res[sw] = rel;
      if (sw >= 16) sweep_res[15] = rel;
      pb->host_sc->rr_true = hs[0];
      if (rel <= o->refine_tol) break;
      if (sw >= max_sweeps) { refine_capped = true; break; }
      // inner BF16 solve z ~ H_bf16^{-1} r
      launch_pcg_init_from64(S16, rd, rpart, S.spmv_nwg, o->tol, o->max_iter, o->check_every, s);
      bf_status r0 = run_solve(S16, true);
      if (r0 != BF_OK) return r0;
      if (pb->host_sc->iter == 0) {
        HIPCHK(c, hipMemcpyAsync(zd, rd, 8 * n3, hipMemcpyDeviceToDevice, s));   // no progress: steepest descent
      } else {
        launch_pcg_flush(S16, s);
        HIPCHK(c, hipMemcpyAsync(zd, S16.x, 8 * n3, hipMemcpyDeviceToDevice, s));
      }
      // p = z - sum_j (z.q_j / p_j.q_j) p_j over the window
      const int nwin = std::min(sweeps, kFcgWindow);
      double* P = Pv(sweeps);
      double* Q = Qv(sweeps);
      HIPCHK(c, hipMemcpyAsync(P, zd, 8 * n3, hipMemcpyDeviceToDevice, s));
      if (nwin > 0) {
        const double* qs[kFcgWindow];
        for (int j = 0; j < nwin; ++j) qs[j] = Qv(sweeps - 1 - j);
        launch_dots64((int)n3, zd, qs, nwin, dpart, dots, s);
        double hz[kFcgWindow];
        HIPCHK(c, hipMemcpyAsync(hz, dots, 8 * nwin, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        for (int j = 0; j < nwin; ++j) {
          const double pqj = pq_hist[(sweeps - 1 - j) % kFcgWindow];
          if (pqj > 0.0) launch_axpy_d((int)n3, -hz[j] / pqj, Pv(sweeps - 1 - j), P, s);
        }
      }
      launch_apply64(S, P, Q, s);
      const double* pr[2] = {rd, Q};
      launch_dots64((int)n3, P, pr, 2, dpart, dots, s);
      double hd[2];
      HIPCHK(c, hipMemcpyAsync(hd, dots, sizeof(hd), hipMemcpyDeviceToHost, s));
      HIPCHK(c, hipStreamSynchronize(s));
      if (!(hd[1] > 0.0)) return fail(c, BF_ERR_NOT_SPD, "refinement direction with p^T H p <= 0");
      pq_hist[sweeps % kFcgWindow] = hd[1];
      launch_axpy_d((int)n3, hd[0] / hd[1], P, xd, s);
      ++sweeps;
    }
    pb->host_sc->bb = bb;
    launch_pcg_finish64(S, pb->Linv.as<double>(), pb->xd.as<double>(), pb->pout.as<double>(),
                        pb->viol_part.as<double>(), nviol, s);
  }
  HIPCHK(c, hipEventRecord(pb->ev[4], s));
  HIPCHK(c, hipMemcpyAsync(p_out, pb->pout.p, 24LL * N, kind_out(mem), s));
  const double refine_rr = pb->host_sc->rr_true, refine_bb = pb->host_sc->bb;
  HIPCHK(c, hipMemcpyAsync(pb->host_sc, S.sc, sizeof(PcgScalars), hipMemcpyDeviceToHost, s));
  int nnzb = 0, hflags = 0;
  HIPCHK(c, hipMemcpyAsync(&nnzb, row_ptr + N, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipMemcpyAsync(&hflags, flags, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  pb->nnzb_last = nnzb;
  pb->stepped = true;
  const PcgScalars& h = *pb->host_sc;
  if (stats) {
    float t01 = 0.f, t12 = 0.f, t23 = 0.f, t34 = 0.f;
    (void)hipEventElapsedTime(&t01, pb->ev[0], pb->ev[1]);
    (void)hipEventElapsedTime(&t12, pb->ev[1], pb->ev[2]);
    (void)hipEventElapsedTime(&t23, pb->ev[2], pb->ev[3]);
    (void)hipEventElapsedTime(&t34, pb->ev[3], pb->ev[4]);
    stats->pcg_iters = total_iters;
    stats->refine_sweeps = sweeps;
    if (bf16)
      stats->rel_residual = refine_bb > 0.0 ? std::sqrt(refine_rr / refine_bb) : 0.0;
    else
      stats->rel_residual = h.bb > 0.0 ? std::sqrt(h.rr_true / h.bb) : 0.0;
    for (int k = 0; k < 16; ++k) stats->sweep_rel_residual[k] = sweep_res[k];
    stats->newton_inf_over_h = h.stat_pinf / pb->dt;
    stats->max_violation = h.stat_viol;
    stats->nnzb = nnzb;
    stats->ms_lin = t01;
    stats->ms_pattern = t12;
    stats->ms_assemble = t23;
    stats->ms_pcg = t34;
    // only launches made before convergence did the full SpMV
    // launches that returned at entry (a system waiting for a residual
    // replacement, or already stopped) take a small fraction of a full SpMV:
    // the average is over launches of at least half the median duration
    const int nt = std::min(timed, ntime);
    std::vector<float> d(nt);
    for (int k = 0; k < nt; ++k) (void)hipEventElapsedTime(&d[k], pb->tev[2 * k], pb->tev[2 * k + 1]);
    std::vector<float> srt(d);
    std::sort(srt.begin(), srt.end());
    const float med = nt > 0 ? srt[nt / 2] : 0.f;
    double tot = 0.0;
    int used = 0;
    for (float v : d)
      if (v >= 0.5f * med) { tot += v; ++used; }
    stats->spmv_timed = used;
    stats->ms_spmv_avg = used > 0 ? tot / used : 0.0;
  }
  // in BF16 mode an inner breakdown only ends that inner solve
  const int sflags = bf16 ? (h.flags & ~FLAG_BREAKDOWN) : h.flags;
  pb->last_breakdown = (sflags & FLAG_BREAKDOWN) && !(hflags & ~FLAG_BREAKDOWN) && !(sflags & ~FLAG_BREAKDOWN);
  if (hflags | sflags) return flags_to_status(c, hflags | sflags);
  c->err.clear();
  if ((!bf16 && h.done == 2 && !h.brk) || refine_capped) {
    c->err = refine_capped ? "refinement reached max_sweeps" : "PCG reached max_iter";
    return BF_WARN_PCG_MAXITER;
  }
  return BF_OK;
}

bf_status bf_get_gradient(bf_problem* pb, double* g_out) {
  if (!pb) return BF_ERR_INVALID_ARG;
  bf_context* c = pb->ctx;
  if (!g_out) return fail(c, BF_ERR_INVALID_ARG, "g_out is NULL");
  if (!pb->stepped) return fail(c, BF_ERR_STATE, "no Newton step has been run");
  std::vector<float> g(3LL * pb->N);
  HIPCHK(c, hipMemcpyAsync(g.data(), pb->grad.p, 12LL * pb->N, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (size_t i = 0; i < g.size(); ++i) g_out[i] = g[i];
  return BF_OK;
}

bf_status bf_get_nnzb(bf_problem* pb, int64_t* nnzb) {
  if (!pb) return BF_ERR_INVALID_ARG;
  if (!nnzb) return fail(pb->ctx, BF_ERR_INVALID_ARG, "nnzb is NULL");
  if (!pb->stepped) return fail(pb->ctx, BF_ERR_STATE, "no Newton step has been run");
  *nnzb = pb->nnzb_last;
  return BF_OK;
}

bf_status bf_get_pattern(bf_problem* pb, int32_t* row_ptr, int32_t* col, int32_t* emap, int32_t* cmap, int32_t* diag) {
  if (!pb) return BF_ERR_INVALID_ARG;
  bf_context* c = pb->ctx;
  if (!pb->stepped) return fail(c, BF_ERR_STATE, "no Newton step has been run");
  hipStream_t s = c->stream;
  const int N = pb->N, T = pb->T, n = pb->n_c;
  const int* rp = pb->row_ptr.as<int>();
  const int* cl = pb->col.as<int>();
  if (row_ptr) HIPCHK(c, hipMemcpyAsync(row_ptr, rp, 4LL * (N + 1), hipMemcpyDeviceToHost, s));
  if (col) HIPCHK(c, hipMemcpyAsync(col, cl, 4LL * pb->nnzb_last, hipMemcpyDeviceToHost, s));
  DevBuf tmp;
  const long long need = 4LL * ((long long)10 * T > 10LL * n ? 10LL * T : 10LL * n) + 4LL * N + 64;
  ALLOC(c, tmp, need);
  if (emap) {
    launch_emap(pb->tets.as<int4>(), T, rp, cl, tmp.as<int>(), s);
    HIPCHK(c, hipMemcpyAsync(emap, tmp.p, 40LL * T, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
  }
  if (cmap && n) {
    launch_cmap(pb->cids.as<int4>(), n, rp, cl, tmp.as<int>(), s);
    HIPCHK(c, hipMemcpyAsync(cmap, tmp.p, 40LL * n, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
  }
  if (diag) {
    launch_row_diag_slots(N, rp, tmp.as<int>(), s);
    HIPCHK(c, hipMemcpyAsync(diag, tmp.p, 4LL * N, hipMemcpyDeviceToHost, s));
  }
  HIPCHK(c, hipStreamSynchronize(s));
  tmp.release();
  return BF_OK;
}

bf_status bf_get_blocks(bf_problem* pb, double* vals) {
  if (!pb) return BF_ERR_INVALID_ARG;
  bf_context* c = pb->ctx;
  if (!vals) return fail(c, BF_ERR_INVALID_ARG, "vals is NULL");
  if (!pb->stepped) return fail(c, BF_ERR_STATE, "no Newton step has been run");
  HIPCHK(c, hipMemcpyAsync(vals, pb->vals.p, 72LL * pb->nnzb_last, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return BF_OK;
}

}  // extern "C"

// ------------------------------------------------------------ subproblem

namespace {

// L(xs) in FP64 (the total energy of Section 4.2 with minimizing slacks);
// *inv is set when some tet of xs is inverted (L is then infinite).
bf_status energy_at(bf_problem* pb, const double* xs, double* L, int* inv, double* ext = nullptr,
                    size_t ext_bytes = 0) {
  bf_context* c = pb->ctx;
  hipStream_t s = c->stream;
  const int np = energy_parts(pb->T, pb->n_c, pb->n_f);
  FrictionView fr;
  fr.n_f = pb->n_f;
  fr.ids = pb->fids.as<int4>();
  fr.f64 = pb->f64.as<double>();
  fr.x0 = pb->fx0.as<double>();
  fr.e = pb->fric_e;
  double* part = ext;
  if (ext) {   // caller's storage: np partials, the sum and the flag
    if (8ULL * (np + 8) > ext_bytes)
      return fail(c, BF_ERR_INVALID_ARG, "problem too large for the no-allocation scratch: the energy needs " +
                                             std::to_string(8ULL * (np + 8)) + " bytes, the scratch holds " +
                                             std::to_string(ext_bytes));
  } else {
    ALLOC(c, pb->epart, 8LL * (np + 8));
    part = pb->epart.as<double>();
  }
  int* flag = reinterpret_cast<int*>(part + np + 2);
  fill_int(flag, 0, 2, s);
  launch_energy(pb->tets.as<int4>(), pb->T, pb->rest.as<double>(), pb->E.as<double>(), pb->nu.as<double>(),
                pb->rho.as<double>(), pb->dt, xs, pb->xt.as<double>(), pb->cids.as<int4>(), pb->n_c,
                pb->lin64.as<double>(), pb->x.as<double>(), pb->clam.as<double>(), pb->cgam.as<double>(), pb->kappa,
                pb->delta, pb->has_mat ? pb->mat.as<int>() : nullptr, fr, part, flag, s);
  launch_sum_to(part, np, part + np, s);
  // part[np] = the sum, part[np + 2] holds the inversion flag (an int)
  double h[3] = {0.0, 0.0, 0.0};
  HIPCHK(c, hipMemcpyAsync(h, part + np, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  int fl = 0;
  std::memcpy(&fl, &h[2], sizeof(int));
  *inv = fl;
  *L = fl ? INFINITY : h[0];
  return BF_OK;
}

}  // namespace

extern "C" {

bf_status bf_energy(bf_problem* pb, double* energy_out, int32_t* inverted) {
  if (!pb) return BF_ERR_INVALID_ARG;
  bf_context* c = pb->ctx;
  if (!energy_out) return fail(c, BF_ERR_INVALID_ARG, "energy_out is NULL");
  if (!pb->stepped) return fail(c, BF_ERR_STATE, "no Newton step has been run (the linearization is missing)");
  HIPCHK(c, hipSetDevice(c->device));
  int inv = 0;
  const bf_status st = energy_at(pb, pb->xh.as<double>(), energy_out, &inv);
  if (inverted) *inverted = inv;
  return st;
}

bf_status bf_energy_noalloc(bf_problem* pb, double* energy_out, int32_t* inverted) {
  if (!pb) return BF_ERR_INVALID_ARG;
  bf_context* c = pb->ctx;
  if (!energy_out) return fail(c, BF_ERR_INVALID_ARG, "energy_out is NULL");
  if (!pb->stepped) return fail(c, BF_ERR_STATE, "no Newton step has been run (the linearization is missing)");
  HIPCHK(c, hipSetDevice(c->device));
  void* ptr = scratch_of(c->device);
  if (!ptr) return fail(c, BF_ERR_HIP, "the scratch of this device was not set up");
  int inv = 0;
  const bf_status st = energy_at(pb, pb->xh.as<double>(), energy_out, &inv, static_cast<double*>(ptr), kScratchBytes);
  if (inverted) *inverted = inv;
  return st;
}

bf_status bf_mu_init(bf_problem* pb, double C, double* mu_out) {
  if (!pb) return BF_ERR_INVALID_ARG;
  bf_context* c = pb->ctx;
  if (!mu_out) return fail(c, BF_ERR_INVALID_ARG, "mu_out is NULL");
  if (!(C > 0.0) || !std::isfinite(C)) return fail(c, BF_ERR_INVALID_ARG, "C must be finite and > 0");
  if (!pb->has_state) return fail(c, BF_ERR_STATE, "bf_set_state must be called first");
  HIPCHK(c, hipSetDevice(c->device));
  hipStream_t s = c->stream;
  const int N = pb->N, T = pb->T;
  int* flags = pb->flags.as<int>();
  fill_int(flags, 0, 16, s);
  // the elastic Hessian at x, the state the time step starts from, into the
  // staging buffer (the next Newton step overwrites it)
  launch_elastic(pb->tets.as<int4>(), T, pb->rest.as<double>(), pb->x.as<double>(), pb->Dminv9.as<double>(),
                 pb->vol.as<float>(), pb->mu.as<float>(), pb->lam.as<float>(), pb->dt * pb->dt,
                 pb->epos.as<int>(), pb->staging.as<double>(), pb->has_mat ? pb->mat.as<int>() : nullptr, flags, s);
  const int np = diag_max_parts(N);
  ALLOC(c, pb->epart, 8LL * (np + 8));
  launch_diag_max(N, pb->erow_ptr.as<int>(), pb->ecptr.as<int>(), pb->staging.as<double>(), pb->mass.as<double>(),
                  pb->epart.as<double>(), s);
  std::vector<double> hp(np);
  HIPCHK(c, hipMemcpyAsync(hp.data(), pb->epart.p, 8LL * np, hipMemcpyDeviceToHost, s));
  int hflags = 0;
  bf_status r0 = read_flags(pb, &hflags);   // synchronizes the stream
  if (r0 != BF_OK) return r0;
  if (hflags) return flags_to_status(c, hflags);
  double m = 0.0;
  for (double v : hp) m = std::max(m, v);
  *mu_out = C * m;
  c->err.clear();
  return BF_OK;
}

bf_status bf_solve_subproblem(bf_problem* pb, const bf_solve_opts* o, int32_t max_newton, double decay,
                              double* x_hat_out, double* lambda_out, double* gamma_out, int32_t mem,
                              bf_subproblem_stats* stats) {
  if (!pb) return BF_ERR_INVALID_ARG;
  bf_context* c = pb->ctx;
  if (!o) return fail(c, BF_ERR_INVALID_ARG, "opts is NULL");
  if (max_newton < 1) return fail(c, BF_ERR_INVALID_ARG, "max_newton must be >= 1");
  if (!(decay > 0.0 && decay <= 1.0)) return fail(c, BF_ERR_INVALID_ARG, "decay must lie in (0, 1]");
  if (mem != BF_MEM_HOST && mem != BF_MEM_DEVICE) return fail(c, BF_ERR_INVALID_ARG, "bad mem kind");
  if (!pb->has_state) return fail(c, BF_ERR_STATE, "bf_set_state must be called first");
  if (pb->cap_nnzb == 0) return fail(c, BF_ERR_STATE, "bf_set_constraints must be called first");
  HIPCHK(c, hipSetDevice(c->device));
  hipStream_t s = c->stream;
  const int N = pb->N, n = pb->n_c;
  const long long n3 = 3LL * N;
  ALLOC(c, pb->pdir, 8 * n3);
  ALLOC(c, pb->xtrial, 8 * n3);
  hipEvent_t e0 = pb->ev[0];
  bf_subproblem_stats out{};
  double* xh = pb->xh.as<double>();
  double L0 = 0.0;
  bool have_L0 = false;
  bf_status warn = BF_OK;
  float total_ms = 0.f;
  for (int it = 0; it < max_newton; ++it) {
    bf_step_stats ns{};
    pb->last_breakdown = false;
    const bf_status st = bf_newton_step(pb, o, pb->pdir.as<double>(), BF_MEM_DEVICE, &ns);
    if (st == BF_ERR_NOT_SPD && pb->last_breakdown) {
      // negative curvature met by the PCG: the iterate reached so far is a
      // descent direction of the quadratic model (truncated Newton); the line
      // search decides how far to go
      ++out.truncated;
      warn = BF_WARN_PCG_MAXITER;
    } else if (st < 0) {
      return st;
    } else if (st > 0) {
      warn = st;
    }
    total_ms += (float)(ns.ms_lin + ns.ms_pattern + ns.ms_assemble + ns.ms_pcg);
    out.pcg_iters += ns.pcg_iters;
    ++out.newton_iters;
    HIPCHK(c, hipEventRecord(e0, s));
    if (!have_L0) {   // the linearization exists from the first step on
      int inv = 0;
      bf_status r0 = energy_at(pb, xh, &L0, &inv);
      if (r0 != BF_OK) return r0;
      ++out.energy_evals;
      if (inv) return fail(c, BF_ERR_INVERTED_ELEMENT, "inverted element in the initial x_hat");
      out.energy_initial = L0;
      have_L0 = true;
    }
    // halving line search: the first r = 2^-k with L(x_hat + r p) < L(x_hat)
    double r = 1.0, L = L0;
    bool ok = false;
    for (int k = 0; k <= 30; ++k, r *= 0.5) {
      launch_state_axpy((int)n3, xh, r, pb->pdir.as<double>(), pb->xtrial.as<double>(), s);
      int inv = 0;
      bf_status r0 = energy_at(pb, pb->xtrial.as<double>(), &L, &inv);
      if (r0 != BF_OK) return r0;
      ++out.energy_evals;
      if (!inv && L < L0) { ok = true; break; }
    }
    if (!ok) r = 0.0;
    if (ok) {
      HIPCHK(c, hipMemcpyAsync(xh, pb->xtrial.p, 8 * n3, hipMemcpyDeviceToDevice, s));
      L0 = L;
    }
    HIPCHK(c, hipEventRecord(pb->ev[1], s));
    HIPCHK(c, hipStreamSynchronize(s));
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, pb->ev[1]);
    total_ms += ms;
    out.last_step = r;
    if (r == 1.0 || r == 0.0) break;
  }
  out.energy_final = L0;
  // multiplier and decay update at the final x_hat
  const int g = div_up(n, 256);
  ALLOC(c, pb->epart, 8LL * (2 * g + 8));
  double* part = pb->epart.as<double>();
  double hc[2] = {0.0, 0.0};
  if (n > 0) {
    launch_dual_update(pb->cids.as<int4>(), n, pb->lin64.as<double>(), pb->x.as<double>(), xh, pb->kappa, pb->delta,
                       decay, pb->clam.as<double>(), pb->cgam.as<double>(), part, s);
    std::vector<double> hp(2 * g);
    HIPCHK(c, hipMemcpyAsync(hp.data(), part, 16LL * g, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    for (int k = 0; k < g; ++k) {
      hc[0] += hp[k];
      hc[1] = std::max(hc[1], hp[g + k]);
    }
  }
  out.active = (int32_t)hc[0];
  out.decayed = n - out.active;
  out.max_violation = hc[1];
  out.ms_total = total_ms;
  if (x_hat_out) HIPCHK(c, hipMemcpyAsync(x_hat_out, xh, 8 * n3, kind_out(mem), s));
  if (lambda_out && n) HIPCHK(c, hipMemcpyAsync(lambda_out, pb->clam.p, 8LL * n, kind_out(mem), s));
  if (gamma_out && n) HIPCHK(c, hipMemcpyAsync(gamma_out, pb->cgam.p, 8LL * n, kind_out(mem), s));
  HIPCHK(c, hipStreamSynchronize(s));
  if (stats) *stats = out;
  c->err.clear();
  return warn;
}

}  // extern "C"
