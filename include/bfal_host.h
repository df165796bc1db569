/* libbfal host rules: the parts of the library that need no device.
 *
 * Argument validation of the descriptors the device entry points take, the
 * penalty stall rule of the time step (Section 5.2), the admission policy of
 * the serving engine and the SpMV's plan of which wavefront takes which
 * slice.  bf_problem_create, bf_set_state,
 * bf_set_constraints, bf_newton_step, bf_time_step and the bf_server_* calls
 * apply exactly these functions; they are exported so that a caller can apply
 * them ahead of a call (a serving front end validating a request before it
 * queues it, a dispatcher over several servers) and so that they run on a
 * machine without a GPU.  Plain C, no allocation except inside
 * bf_admission_create/push, no HIP call anywhere.
 *
 * Messages: every bf_check_* writes a NUL-terminated reason into msg (at most
 * msg_cap bytes, truncated) when it returns an error; msg may be NULL.
 */
#ifndef BFAL_HOST_H
#define BFAL_HOST_H

#include "bfal.h"

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ validation --
 * Host-memory descriptors only (the device-pointer path checks contents in
 * its kernels and reports through the same status codes).
 *
 * bf_check_mesh: the arrays are non-NULL, n_nodes and n_tets positive and
 * small enough for 32-bit slot indices (10 T and 3 N below 2^31), every tet
 * vertex in [0, n_nodes) and the four distinct, E > 0, -1 < nu < 0.5, rho > 0
 * (finite), material codes in {0, 1, 2} when given, finite rest positions.
 * Returns BF_OK or BF_ERR_INVALID_ARG. */
bf_status bf_check_mesh(const bf_mesh_desc* m, char* msg, int32_t msg_cap);

/* bf_check_state: the three [n_nodes][3] arrays are non-NULL and finite and
 * dt > 0 is finite (the incremental potential of Section 3 needs a positive
 * step).  Returns BF_OK or BF_ERR_INVALID_ARG. */
bf_status bf_check_state(int32_t n_nodes, const double* x, const double* x_hat, const double* x_tilde, double dt,
                         char* msg, int32_t msg_cap);

/* bf_check_constraints: the constraint set C = {(i, lambda_i, gamma_i)} of
 * Algorithm 2 with the penalty kappa > 0 and offset delta >= 0 (Section 4.2):
 * counts non-negative and below 2^31 / 10 together, arrays present for every
 * non-empty part, indices in [0, n_nodes), lambda finite and >= 0, gamma in
 * (0, 1] when given.  Returns BF_OK, BF_ERR_INVALID_ARG, or
 * BF_ERR_DEGENERATE_CONSTRAINT for a row with a repeated vertex (its
 * distance has no unique gradient). */
bf_status bf_check_constraints(int32_t n_nodes, const bf_constraint_desc* cd, char* msg, int32_t msg_cap);

/* bf_check_solve_opts: tol > 0 (the CG relative tolerance of Section 6),
 * max_iter >= 0, a known precision mode, refine_tol > 0 in the BF16 mode.
 * Returns BF_OK or BF_ERR_INVALID_ARG. */
bf_status bf_check_solve_opts(const bf_solve_opts* o, char* msg, int32_t msg_cap);

/* ------------------------------------------------------------ stall rule --
 * Section 5.2: when the step size alpha of the outer loop (Algorithm 1)
 * stays below alpha_min for `window` consecutive iterations, the penalty
 * doubles and the offset delta halves; the count then restarts.  The time
 * step uses alpha_min = 1e-4 and window = 50.  Start with count = 0. */
typedef struct {
  double alpha_min;
  int32_t window;
  int32_t count; /* consecutive iterations below alpha_min so far */
} bf_stall_rule;

/* Feed the alpha of one outer iteration.  Returns 1 (and doubles *kappa,
 * halves *delta) when the window fills, else 0.  -1 on a NULL argument or a
 * window < 1. */
int32_t bf_stall_step(bf_stall_rule* rule, double alpha, double* kappa, double* delta);

/* ------------------------------------------------------------- admission --
 * Admission policy of the serving engine: requests wait in arrival order;
 * the head is admitted when a slot is free and its device footprint
 * (bf_footprint_bytes) fits beside the admitted ones in the budget; a
 * request that could never fit (footprint > budget) is rejected at the head
 * without blocking the queue (the server reports BF_ERR_BUDGET for it).
 * Not thread-safe: the server calls it under its own lock. */
typedef struct bf_admission bf_admission;

bf_status bf_admission_create(uint64_t hbm_budget, int32_t slots, bf_admission** out);
void bf_admission_destroy(bf_admission* a);
/* Queue request `id` with its footprint.  BF_ERR_OOM if the queue cannot grow. */
bf_status bf_admission_push(bf_admission* a, int64_t id, uint64_t footprint);
/* Decide on the head of the queue: returns 1 and sets *id, *slot when it is
 * admitted (its footprint now counts against the budget and the slot is
 * taken), -1 and sets *id when it is rejected as never fitting (removed from
 * the queue), 0 when the queue is empty or the head must wait. */
int32_t bf_admission_next(bf_admission* a, int64_t* id, int32_t* slot);
/* A request admitted into `slot` with `footprint` finished: free both.
 * BF_ERR_INVALID_ARG if the slot is not in use or the footprint does not
 * match what was admitted into it. */
bf_status bf_admission_release(bf_admission* a, int32_t slot, uint64_t footprint);
/* Bytes admitted now, requests waiting, slots in use. */
uint64_t bf_admission_used(const bf_admission* a);
int32_t bf_admission_waiting(const bf_admission* a);
int32_t bf_admission_active(const bf_admission* a);

/* ------------------------------------------------------ SpMV slice plan --
 * Which slices of the sliced matrix storage each SpMV wavefront processes.
 * The SpMV gives one 64-row slice at a time to a wavefront; its workgroups
 * are spread over the device's 8 XCDs (accelerator complex dies), each with
 * its own L2, workgroup w of `nparts / 4` on XCD w / (nparts / 32) and wave v
 * of it taking part 4 w + v.  A slice's cost is ceil(max(wu, wl) / pairs) + 1
 * steps, wu and wl its upper and lower slot widths ((slot_u[s+1] - slot_u[s])
 * / 64 and the same for slot_l, the exclusive scans of 64 x the widths).
 * The plan keeps the slices that are read together on one XCD and balances
 * the parts: the slices are cut into 8 consecutive windows of equal cost
 * (window x to XCD x; window x starts at the first slice whose cost prefix
 * reaches x / 8 of the total); each window is taken in consecutive blocks of
 * 2 nparts / 8 slices, and inside a block the slices, costliest first (ties
 * in slice order), go one by one to the part of that XCD with the least cost
 * so far (the lowest index on ties).  Each XCD thus sweeps its window from
 * start to end, two slices per part per block.  Output as lists:
 * part p takes wave_slices[wave_ptr[p] .. wave_ptr[p+1]), increasing.
 *   nslices >= 1; slot_u, slot_l: [nslices + 1] nondecreasing multiples of 64;
 *   pairs >= 1 (upper/lower pairs per SpMV step); nparts: a positive multiple
 *   of 8; wave_ptr: [nparts + 1]; wave_slices: [nslices] (caller-owned).
 * Returns BF_ERR_INVALID_ARG for a NULL array, a size out of range or slot
 * offsets that are not nondecreasing multiples of 64 (nothing written then),
 * BF_ERR_OOM if the host cannot allocate the per-part costs, else BF_OK.
 * Every slice is listed exactly once. */
bf_status bf_slice_plan(int32_t nslices, const int32_t* slot_u, const int32_t* slot_l, int32_t pairs,
                        int32_t nparts, int32_t* wave_ptr, int32_t* wave_slices);

#ifdef __cplusplus
}
#endif

#endif /* BFAL_HOST_H */
