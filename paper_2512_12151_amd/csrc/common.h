// Internal declarations shared by the host orchestration and the kernels of
// libbfal.  Nothing here is part of the C-ABI (see include/bfal.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <string>

#include "../../include/bfal.h"

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
  double rho;        // r^T r of the scaled system (= r^T M^{-1} r of the original)
  double pp;         // p^T p
  double pq;         // p^T H p
  double alpha, beta;
  double rr_true;    // |L r|^2 = unscaled residual norm squared (when checked)
  double bb;         // |b|^2 (unscaled)
  double tol2;       // tol^2
  double stat_pinf;  // max |p_i| of the result
  double stat_viol;  // max_i max(0, -c_i)
  int iter2;         // iteration index seen by the update kernel (written by its workgroup 0)
  int iter3;         // completed iterations (written by workgroup 0 of the direction kernel)
  int done;          // 1: converged, 2: max_iter, 3: breakdown
  int max_iter;
  int check_every;
  int flags;         // FLAG_* bits
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
// Sort every segment [ptr[i], ptr[i+1]) of keys ascending (thread per segment).
void sort_segments(int* keys, const int* ptr, int nseg, hipStream_t s);
void fill_int(int* a, int v, long long n, hipStream_t s);

// setup.hip: per-mesh work
void launch_check_tets(const int4* tets, int T, int N, int* flags, hipStream_t s);
void launch_rest_geometry(const int4* tets, const double* rest, const double* E, const double* nu,
                          int T, float* Dminv9, float* vol, float* mu, float* lam, int* flags,
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
                 const double* rho, int N, float* mass, hipStream_t s);

// contact.hip: per-step constraint work
void launch_check_constraints(const int4* ids, int n_c, int N, const double* lam, const double* gam,
                              int* flags, hipStream_t s);
void launch_contact_lin(const int4* ids, int n_pt, int n_c, const double* x, const double* xh,
                        const double* lam, const double* gam, double kappa, double delta,
                        float* cn, float* cw, float* cg, float* ch, double* viol_part, int* flags,
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

// elastic.hip
void launch_elastic(const int4* tets, int T, const double* rest, const double* xh, const float* Dminv9,
                    const float* vol, const float* mu, const float* lam, float h2, const int* epos,
                    float* staging, int* flags, hipStream_t s);

// assemble.hip
void launch_assemble_rows(int N, const int* row_ptr, const int* col, const int* eslot, const int* ecptr,
                          const float* staging, const int* vptr, const int* vinc, const int4* ids, int n_c,
                          const float* cn, const float* cw, const float* cg, const float* ch,
                          const float* mass, const double* xh, const double* xt, const uint8_t* fixed,
                          float* vals, float* grad, float* Lf, float* Linv, float* bhat, double* bb_part,
                          int* flags, hipStream_t s);
// Scaled upper off-diagonal blocks as SoA [9][stride] and the transpose index
// (lower_count / lower_fill / sort_segments give, per column, the source rows;
// transpose_index turns them into upper block indices).
void launch_lower_count(int N, const int* row_ptr, const int* col, int* lcnt, hipStream_t s);
void launch_lower_fill(int N, const int* row_ptr, const int* col, const int* lptr, int* lcur, int* lsrc,
                       hipStream_t s);
void launch_scale_upper(int N, const int* row_ptr, const int* col, const float* vals, const float* Linv, float* uvals,
                        int* ucol, int* urow_ptr, long long ustride, hipStream_t s);
void launch_transpose_index(int N, const int* row_ptr, const int* col, const int* lptr, const int* lsrc, int* tidx,
                            hipStream_t s);
void launch_row_diag_slots(int N, const int* row_ptr, int* diag, hipStream_t s);

// pcg.hip
int pcg_partials_needed(int N);
void launch_pcg_init(int N, const float* bhat, float* x, float* r, float* p, double* part,
                     const double* bb_part, int nbb, PcgScalars* sc, double tol, int max_iter,
                     int check_every, hipStream_t s);
// One PCG iteration = launch_pcg_spmv then launch_pcg_vector_ops (update + direction).
// The SpMV's first phase writes q_row = p + (upper part) p and, for every upper
// block j, its transposed product B_j^T p_r into tbuf; launch_pcg_vector_ops
// completes q = q_row + sum of tbuf over the transpose index, then updates.
void launch_pcg_spmv(int N, const int* urow_ptr, const int* ucol, const float* uvals, long long ustride,
                     const float* p, float* qrow, float* tbuf, double* part, PcgScalars* sc, hipStream_t s);
void launch_pcg_vector_ops(int N, const float* Lf, float* x, float* r, float* p, const float* qrow,
                           const float* tbuf, const int* tptr, const int* tidx, double* part, PcgScalars* sc,
                           hipStream_t s);
void launch_pcg_finish(int N, const float* Linv, const float* x, double* pout, double* part,
                       PcgScalars* sc, const double* viol_part, int nviol, hipStream_t s);

}  // namespace bfal
