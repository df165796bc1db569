// Internal declarations shared by the host orchestration and the kernels of
// libbfal.  Nothing here is part of the C-ABI (see include/bfal.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <string>

#include "../../include/bfal.h"
#include "../../include/bfal_host.h"

namespace bfal {

// Error bits raised by kernels into a device word and mapped to bf_status by
// the host after the step.
enum : int {
  FLAG_INVERTED = 1,     // det F <= 0 in some tet
  FLAG_DEGENERATE = 2,   // d_i(x) <= 0 or a (near-)parallel EE pair
  FLAG_NOT_SPD = 4,      // a diagonal block failed its Cholesky factorization
  FLAG_BAD_INDEX = 8,    // a device-resident index array held an out-of-range id
  FLAG_BREAKDOWN = 16,   // p^T H p <= 0 inside PCG
  FLAG_BAD_VALUE = 32,   // non-finite or out-of-range device-resident value
};

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kBlock = 256;        // default workgroup size (4 waves)

// Device-resident scalars of one PCG solve (see pcg.hip for who writes what).
struct PcgScalars {
  // Control words first, grouped so that each PCG kernel reads its own in one
  // load and none of them reads a word it writes: the update kernel reads
  // [ks, done, check_every, xbase], the SpMV [check_every, xbase, iter, brk].
  int ks;            // iteration index of the last SpMV (written by its workgroup 0)
  int done;          // 1: converged, 2: max_iter, 4: residual replacement requested
                     // (written by workgroup 0 of the SpMV; cleared by the replacement)
  int check_every;
  int xbase;         // x holds alpha_j p_j for every j < xbase and for every j below the last multiple of kXBatch
                     // reached by the update kernel (written by the flush kernel only)
  int iter;          // completed iterations (written by workgroup 0 of the update kernel)
  int brk;           // 1: breakdown p^T H p <= 0 (written by workgroup 0 of the update kernel)
  int max_iter;
  int verified;      // iteration of the last residual replacement (-1: none)
  int replace_on;    // 1: replace the residual (see pcg.hip), 0: plain recurrences
  int flags;         // FLAG_* bits
  double rho;        // r^T r of the scaled system (= r^T D^{-1} r of the original)
  double rr_true;    // |L r|^2 = unscaled residual norm squared (when checked)
  double bb;         // |b|^2 (unscaled)
  double tol2;       // tol^2
  double stat_pinf;  // max |p_i| of the result
  double stat_viol;  // max_i max(0, -c_i)
  double rt_ref;     // |L r|^2 right after the last residual replacement (or |b|^2)
  float alpha_hist[8];   // alpha_j at j % kXBatch (written by workgroup 0 of the update kernel)
};

// x += alpha_j p_j is applied kXBatch iterations at a time (the update kernel
// of every kXBatch-th iteration, or a flush before x is read): the directions
// p_j live in a ring of kPRing buffers until then.
constexpr int kXBatch = 8;
constexpr int kPRing = kXBatch + 1;

// Partials of one PCG system: every workgroup writes one FP64 value per sum.
constexpr int kMaxVecParts = 1024;    // workgroups of the update kernel per system
constexpr int kMaxSpmvParts = 2048;   // workgroups of the SpMV per system
constexpr int kPartRR = 0;                              // r^T r, two slots (iterations k, k+1)
constexpr int kPartRT = 2 * kMaxVecParts;               // |L r|^2
constexpr int kPartPQ = 3 * kMaxVecParts;               // p^T H p
constexpr int kPartRQ = kPartPQ + kMaxSpmvParts;        // r^T H p
constexpr int kPartQQ = kPartRQ + kMaxSpmvParts;        // |H p|^2
constexpr int kPartsPerSystem = 3 * kMaxVecParts + 3 * kMaxSpmvParts;

constexpr int kSlice = 64;         // rows per slice of the sliced block storage (one wavefront)

// One symmetric block system of the PCG, H_hat = L^{-1} H L^{-T} with identity
// diagonal blocks, in sliced storage (kSlice consecutive rows per slice, slot k
// of the row in lane l of slice s at sbu[s] + k * kSlice + l):
//   upper slots  blk (FP32 9 floats, or BF16 5 words) and scol: the upper
//                off-diagonal blocks of the row and their columns;
//   lower slots  sent = (upper slot, source row r) of every upper block (r, c)
//                of the row's column c, by increasing r;
// padded slots hold a zero block, and zeroed padding follows the last slot of
// each array (see slot_padding).  Vectors are FP32 AoS [N4][3] (N4 = N
// rounded up to 4; pads are zero), Lf is SoA [6][N4].  The SpMV grid gives this
// system spmv_nwg workgroups of 4 slices each; the update grid vec_nwg.
struct PcgSystem {
  int N, N4, nslices;
  const int* sbu;    // [nslices + 1]
  const int* sbl;    // [nslices + 1]
  const int* wave_ptr;     // SpMV slice plan (bf_slice_plan for 4 * spmv_nwg parts): part p takes
  const int* wave_slices;  // wave_slices[wave_ptr[p] .. wave_ptr[p + 1])
  const int* scol;
  const void* blk;
  const int2* sent;
  const float* Lf;
  double* x;         // FP64 solution (AoS [N4][3])
  float* r;
  float* P;          // ring of kPRing direction buffers: p_k at P + (k % kPRing) * pstride
  long long pstride; // floats per direction buffer (3 N4)
  float* q;
  double* part;      // kPartsPerSystem
  PcgScalars* sc;
  int spmv_wg0, spmv_nwg;
  int vec_wg0, vec_nwg;
};

__host__ __device__ inline int div_up(long long a, long long b) { return (int)((a + b - 1) / b); }

// A growable device buffer.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  hipError_t ensure(size_t n) {
    if (n <= bytes && p) return hipSuccess;
    if (p) { hipError_t e = hipFree(p); p = nullptr; bytes = 0; if (e != hipSuccess) return e; }
    size_t want = n ? n : 16;
    hipError_t e = hipMalloc(&p, want);
    if (e == hipSuccess) bytes = want;
    return e;
  }
  void release() { if (p) (void)hipFree(p); p = nullptr; bytes = 0; }
  template <class T> T* as() const { return static_cast<T*>(p); }
};

// ----------------------------------------------------------- kernel entry
// Each .hip file exposes host launchers; all take the stream last.

// scan.hip: exclusive prefix sum of n ints; out may alias in; *total (device)
// receives the sum.  tmp must hold scan_tmp_ints(n) ints.
size_t scan_tmp_ints(long long n);
void scan_exclusive(const int* in, int* out, long long n, int* total, int* tmp, hipStream_t s);
// Sort every segment [ptr[i], ptr[i+1]) of keys ascending (a wavefront per segment; stable).
void sort_segments(int* keys, const int* ptr, int nseg, hipStream_t s);
void fill_int(int* a, int v, long long n, hipStream_t s);

// setup.hip: per-mesh work
void launch_check_tets(const int4* tets, int T, int N, int* flags, hipStream_t s);
void launch_rest_geometry(const int4* tets, const double* rest, const double* E, const double* nu,
                          const double* rho, int T, double* Dminv9, float* vol, float* mu, float* lam, int* flags,
                          hipStream_t s);
void launch_elastic_pair_count(const int4* tets, int T, int* cnt, hipStream_t s);
void launch_elastic_pair_fill(const int4* tets, int T, const int* ptr, int* cursor, int* keys,
                              hipStream_t s);
void launch_row_unique(int* keys, const int* kptr, int N, int* ucount, hipStream_t s);
void launch_row_write(const int* keys, const int* kptr, int N, const int* row_ptr, int* col, hipStream_t s);
void launch_emap(const int4* tets, int T, const int* row_ptr, const int* col, int* emap, hipStream_t s);
void launch_slot_count(const int* map, long long n, int* cnt, hipStream_t s);
void launch_slot_fill(const int* map, long long n, const int* ptr, int* cursor, int* list, hipStream_t s);
void launch_inverse_positions(const int* list, long long n, int* pos, hipStream_t s);
void launch_mass(const int* ecptr, const int* elist, const int* erow_ptr, const float* vol,
                 const double* rho, int N, double* mass, hipStream_t s);

// contact.hip: per-step constraint work
void launch_check_constraints(const int4* ids, int n_c, int N, const double* lam, const double* gam,
                              int* flags, hipStream_t s);
// lin64 receives the linearization, SoA [8][n_c]: d, n (3), w (4); cg and ch
// the gradient factor kappa gamma (c - lambda / kappa - s) and the Hessian
// factor kappa gamma of each constraint.
void launch_contact_lin(const int4* ids, int n_pt, int n_c, const double* x, const double* xh,
                        const double* lam, const double* gam, double kappa, double delta,
                        double* cg, double* ch, double* lin64, double* viol_part, int* flags,
                        hipStream_t s);
void launch_vertex_incidence_count(const int4* ids, int n_c, int* cnt, hipStream_t s);
void launch_vertex_incidence_fill(const int4* ids, int n_c, const int* ptr, int* cursor, int* inc,
                                  hipStream_t s);
void launch_candidate_count(const int* erow_ptr, const int* vptr, const int* vinc, const int4* ids,
                            int N, int* ccount, hipStream_t s);
void launch_candidate_fill(const int* erow_ptr, const int* ecol, const int* vptr, const int* vinc,
                           const int4* ids, int N, const int* cptr, int* cand, int* ucount,
                           hipStream_t s);
void launch_merged_write(const int* cand, const int* cptr, const int* row_ptr, const int* erow_ptr,
                         const int* ecol, int N, int* col, int* eslot, hipStream_t s);
void launch_cmap(const int4* ids, int n_c, const int* row_ptr, const int* col, int* cmap, hipStream_t s);

// subproblem.hip (the rest of Algorithm 2).  The total energy L(x) in FP64
// (per-tet Neo-Hookean from the rest shape, lumped inertia folded per tet,
// slack-minimized AL terms from lin64) as nparts partials in part, and any
// inverted tet raised into *inverted; xt = xa + r p; the multiplier and
// decay update in place (counts of active constraints and the violation
// max into per-workgroup partials).
// The friction set of a step (Appendix A): contacts, the FP64 capture SoA
// [8][n_f] (normal, weights, coefficient), x^t and e = eps_v h.
struct FrictionView {
  int n_f = 0;
  const int4* ids = nullptr;
  const double* f64 = nullptr;
  const double* x0 = nullptr;
  double e = 0.0;
};
int energy_parts(int T, int n_c, int n_f);
void launch_energy(const int4* tets, int T, const double* rest, const double* E, const double* nu,
                   const double* rho, double h, const double* x, const double* xt, const int4* ids, int n_c,
                   const double* lin64, const double* xlin, const double* lam, const double* gam, double kappa,
                   double delta, const int* mat, FrictionView fr, double* part, int* inverted, hipStream_t s);
void launch_state_axpy(int n3, const double* xa, double r, const double* p, double* xt, hipStream_t s);
// ccd.hip: collision queries along x -> x_hat (boxes are 24-byte FP32 min/max).
size_t ccd_sort_tmp_bytes(int n);
hipError_t ccd_sort_pairs(void* tmp, size_t tmp_bytes, const unsigned long long* kin, unsigned long long* kout,
                          const int* vin, int* vout, int n, hipStream_t s);
size_t ccd_sort_keys_tmp_bytes(int n);
hipError_t ccd_sort_keys(void* tmp, size_t tmp_bytes, const unsigned long long* kin, unsigned long long* kout, int n,
                         hipStream_t s);
void launch_prim_boxes(int n, const int* ids, int k, const double* x, const double* xh, void* box, hipStream_t s);
int ccd_bounds_parts(int n);
void launch_morton(int n, const void* box, void* part, unsigned long long* key, hipStream_t s);
int ccd_table_levels(int n);
void launch_build_tree(int n, const unsigned long long* key, const void* pbox, int2* child, int2* range, void* node,
                       void* table, hipStream_t s);
void launch_query(bool ee, int nq, const int* qids, int nt, const int* tids, const int2* child, const void* node,
                  const unsigned long long* key, const double* x, const double* xh, double delta, double sep,
                  int* count, int cap, int2* pairs, double* toc, hipStream_t s);
void launch_pair_keys(int n, const int2* pairs, unsigned long long* key, int* idx, hipStream_t s);
void launch_hash_insert(int n_c, int n_pt, const int4* ids, int* table, unsigned int mask, hipStream_t s);
void launch_fill_u64(unsigned long long* a, unsigned long long v, int n, hipStream_t s);
void launch_pair_rows(int n, bool ee, const int2* pairs, const int* qids, const int* tids, int4* rows, hipStream_t s);
void launch_new_and_tv(int n, bool ee, const int* order, const int2* pairs, const double* toc, const int* qids,
                       const int* tids, int n_pt, const int4* cids, const int* table, unsigned int mask,
                       const double* x, int* is_new, unsigned long long* tv, hipStream_t s);
void launch_keep_new(int n, bool ee, const int* order, const int2* pairs, const double* toc, const int* qids,
                     const int* tids, const unsigned long long* tv, int* keep, hipStream_t s);
void launch_keep_current(int lo, int hi, const double* gam, double gmin, int* keep, hipStream_t s);
void launch_scatter_current(int lo, int hi, const int* keep, const int* pos, int base, const int4* ids,
                            const double* lam, const double* gam, int4* oids, double* olam, double* ogam,
                            hipStream_t s);
void launch_scatter_new(int n, bool ee, const int* keep, const int* pos, int base, const int* order,
                        const int2* pairs, const int* qids, const int* tids, int4* oids, double* olam, double* ogam,
                        hipStream_t s);
int ccd_min_parts(int n);
void launch_min_toc(int n, const double* toc, double* part, hipStream_t s);
int inversion_parts(int T);
void launch_inversion_bound(int T, const int4* tets, const double* x, const double* xh, double sep, double* part,
                            hipStream_t s);

void launch_blend(int n3, double* x, const double* xh, double alpha, hipStream_t s);
void launch_velocity(int n3, const double* x, const double* x0, double inv_h, double* v, hipStream_t s);
int diag_max_parts(int N);
void launch_diag_max(int N, const int* erow_ptr, const int* ecptr, const double* staging, const double* mass,
                     double* part, hipStream_t s);
void launch_dual_update(const int4* ids, int n_c, const double* lin64, const double* xlin, const double* xh,
                        double kappa, double delta, double decay, double* lam, double* gam, double* part,
                        hipStream_t s);

// contact.hip: semi-implicit friction (capture at x^t into FP64 SoA [8][n_f];
// per-step terms at x_hat into FP64 SoA [13][n_f])
void launch_friction_capture(const int4* ids, int n_pt, int n_f, const double* x, const double* lam, double kappa,
                             double delta, double mu_f, double* f64, hipStream_t s);
void launch_friction_terms(const int4* ids, int n_f, const double* xh, const double* x0, const double* f64, double e,
                           double* fgk, hipStream_t s);
// Friction contact -> constraint with the same stencil: table insert of the
// constraint rows (tab filled with -1 first, mask = capacity - 1), match
// (cfr[ci] = fi, cfr filled with -1 first; extra[fi] = 1 when unmatched), and
// the unmatched contacts' stencils at pids[n_c + pos[fi]] with fext[pos[fi]] = fi.
void launch_stencil_insert(const int4* ids, int n_c, int* tab, unsigned mask, hipStream_t s);
void launch_friction_match(const int4* fids, int n_f, const int4* ids, const int* tab, unsigned mask, int* cfr,
                           int* extra, hipStream_t s);
void launch_friction_extra(const int4* fids, int n_f, const int* extra, const int* pos, int n_c, int4* pids,
                           int* fext, hipStream_t s);

// elastic.hip
void launch_elastic(const int4* tets, int T, const double* rest, const double* xh, const double* Dminv9,
                    const float* vol, const float* mu, const float* lam, double h2, const int* epos,
                    double* staging, const int* mat, int* flags, hipStream_t s);

// assemble.hip
// Off-diagonal elastic sums (one thread per slot of the merged pattern, cap
// >= its slot count), then the row owners (one thread per row).
void launch_assemble_rows(int N, long long cap, const int* row_ptr, const int* col, const int* eslot,
                          const int* erow_ptr, const int* ecol, const int* ecptr, const double* staging,
                          const int* vptr, const int* vinc, const int4* ids, const int* cslot, int n_c,
                          const double* lin64,
                          const double* cg, const double* ch, int n_f, const double* fgk, const int* cfr,
                          const int* fext, const double* mass, const double* xh, const double* xt,
                          const uint8_t* fixed, double* vals, float* grad, float* Lf, double* Linv, float* bhat,
                          double* bb_part, int* flags, hipStream_t s);
// Sliced storage of the scaled matrix: lower_count / lower_fill /
// sort_segments give, per column, the source rows of its upper blocks;
// slice_widths gives the slot counts per slice (64 x the widest row), whose
// exclusive scans are sbu / sbl; sell_fill writes the upper slots (FP32 and,
// when blk16 is set, BF16) and the lower references.
void launch_lower_count(int N, const int* row_ptr, const int* col, int* lcnt, hipStream_t s);
void launch_lower_fill(int N, const int* row_ptr, const int* col, const int* lptr, int* lcur, int* lsrc,
                       hipStream_t s);
void launch_slice_widths(int N, int nslices, const int* row_ptr, const int* lptr, int* cu, int* cl, int* wmax,
                         hipStream_t s);
// The SpMV visits upper and lower slots in pairs, kPairs per step, and reads
// up to (max width + kPairs) * kSlice slots past the end of a slice's range;
// the slot arrays carry that much zeroed padding after their last slot.
constexpr int kPairs = 2;
constexpr int kSpmvWaves = 4;   // wavefronts (slices in flight) per SpMV workgroup
inline long long slot_padding(int wmax_other) { return (long long)(wmax_other + kPairs + 1) * kSlice; }
void launch_sell_fill(int N, int nslices, const int* row_ptr, const int* col, const double* vals, const double* Linv,
                      const int* lptr, const int* lsrc, const int* sbu, const int* sbl, float* blk, uint32_t* blk16,
                      int* scol, int2* sent, hipStream_t s);
void launch_row_diag_slots(int N, const int* row_ptr, int* diag, hipStream_t s);

// pcg.hip
// Workgroup counts of one system.
int pcg_spmv_groups(int N, int num_cu);
int pcg_vec_groups(int N);
// x = 0, r = b_hat, |b|^2 from the assembly's partials, scalars reset.
// replace: enable residual replacement (needs the FP32 blocks in S.blk).
void launch_pcg_init(const PcgSystem& S, const float* bhat, const double* bb_part, int nbb, double tol, int max_iter,
                     int check_every, bool replace, hipStream_t s);
// Residual replacement requested by a system (done == 4): r = b_hat - H_hat x
// in FP64 (rd scratch [3 N4], rpart scratch [kMaxSpmvParts]) rounded to FP32,
// its partials in place of the recursive ones, done cleared.
void launch_pcg_replace(const PcgSystem& S, const float* bhat, double* rd, double* rpart, hipStream_t s);
// One PCG iteration of one system: the SpMV kernel (direction p = r + beta p
// fused in, q = H_hat p, p^T q) then the update kernel (x, r, r^T r, |L r|^2).
// bf16 selects the BF16 block copy.
// With t0 and t1 set, the SpMV dispatch is timed between them.
void launch_pcg_iteration(const PcgSystem& S, bool bf16, hipStream_t s, hipEvent_t t0 = nullptr,
                          hipEvent_t t1 = nullptr);
// The same iteration for several systems in one launch pair: sys[] (device)
// lists them, wg_sys_spmv / wg_sys_vec map each workgroup to its system.
void launch_pcg_iteration_batched(const PcgSystem* sys, const int* wg_sys_spmv, int nwg_spmv, const int* wg_sys_vec,
                                  int nwg_vec, bool bf16, hipStream_t s);
// x += the directions the update kernel has not applied yet (before x is read).
void launch_pcg_flush(const PcgSystem& S, hipStream_t s);
// p = L^{-T} x in FP64 and the stats (max |p|, max violation).
void launch_pcg_finish(const PcgSystem& S, const double* Linv, double* pout, const double* viol_part, int nviol,
                       hipStream_t s);
// Iterative refinement around BF16 inner solves: rd = b_hat - H_hat xd in FP64
// with the FP32 blocks (S.blk must be the FP32 storage), partials of |L rd|^2
// into rpart[spmv_nwg] and their sum into *rsum; an inner solve started from
// rd with bb = the sum of rpart; xd += the inner solution; p = L^{-T} xd.
void launch_residual64(const PcgSystem& S, const float* bhat, const double* xd, double* rd, double* rpart,
                       double* rsum, hipStream_t s);
void launch_sum_to(const double* part, int n, double* out, hipStream_t s);
void launch_pcg_init_from64(const PcgSystem& S, const double* rd, const double* rpart, int nparts, double tol,
                            int max_iter, int check_every, hipStream_t s);
void launch_axpy64(const PcgSystem& S, double* xd, hipStream_t s);
// Outer flexible-CG pieces (FP64 vectors of 3 * N4): yd = H_hat xd (FP32
// blocks, FP64 sums); out[j] = a . b[j] for nb <= 6 vectors (part holds
// 6 * 256 partials); y += alpha x; y = (double) x.
void launch_apply64(const PcgSystem& S, const double* xd, double* yd, hipStream_t s);
void launch_dots64(int n3, const double* a, const double* const* b, int nb, double* part, double* out,
                   hipStream_t s);
void launch_axpy_d(int n3, double alpha, const double* x, double* y, hipStream_t s);
void launch_copy_f2d(int n3, const float* x, double* y, hipStream_t s);
void launch_pcg_finish64(const PcgSystem& S, const double* Linv, const double* xd, double* pout,
                         const double* viol_part, int nviol, hipStream_t s);

}  // namespace bfal
