/*
 * bfal.h -- C-ABI of libbfal: one Newton step of the barrier-free
 * augmented-Lagrangian (AL) contact subproblem on one MI355X (gfx950).
 *
 * The operation (paper: Algorithm 2, the body of the Newton loop; Section 4.2
 * "Augmented Lagrangian-based Subproblem Solver"):
 *
 *   G = grad E(x_hat, x_tilde) + sum_i kappa*gamma_i*(c_i - lambda_i/kappa - s_i) grad d_i(x)
 *   H = SPDProject(hess E(x_hat, x_tilde)) + sum_i kappa*gamma_i grad d_i(x) grad d_i(x)^T
 *   p = -H^{-1} G                     (block-Jacobi preconditioned CG)
 *
 * with E the incremental potential 1/2|x - x_tilde|_M^2 + h^2 U(x) of Section 3
 * (lumped mass M; U on linear tetrahedra of Neo-Hookean, stable Neo-Hookean or
 * corotated linear material per tet (Table 2), plus, after bf_set_friction,
 * the semi-implicit friction potential of Appendix A), the linearized
 * constraints c_i(x_hat) = d_i(x) + grad d_i(x)^T (x_hat - x) - delta of
 * Section 4.2, slacks s_i = max(0, c_i - lambda_i/kappa), the per-element
 * SPD projection of Section 5.1 (eigenvalues of d2Psi/dF2 clamped at zero),
 * and moving-boundary (Dirichlet) nodes eliminated as in Section 5.3.  Around
 * the step the library also runs the rest of SolveSubproblem (Algorithm 2),
 * the collision queries of UpdateActiveSet and MaxStepSize (Algorithms 3, 1)
 * and whole time steps (Algorithm 1), and serves batches of steps.  The
 * paper calls the penalty mu; this ABI calls it kappa to keep mu for the Lame
 * parameter.  d_i is the unsigned distance of a point-triangle (PT) or
 * edge-edge (EE) pair (Section 3).
 *
 * Conventions shared by every call:
 *  - Status: every call returns a bf_status.  Negative values are errors and
 *    leave the outputs unspecified; positive values are warnings and the
 *    outputs are written.  Calls never throw and never abort across the ABI.
 *    bf_last_error() returns a message for the last failing call on a context.
 *  - Memory: array arguments are plain pointers.  `mem` says where they live:
 *    BF_MEM_HOST (pageable or pinned host memory) or BF_MEM_DEVICE (device
 *    memory of the context's GPU, ordered on the context's stream).  Inputs
 *    are borrowed for the duration of the call and copied; outputs are
 *    caller-allocated.  Handles are owned by the caller and freed by the
 *    matching _destroy call.  A context (and its problems) must be used from
 *    one thread at a time.
 *  - Layouts: node arrays are [n_nodes][3] row-major doubles; index arrays are
 *    [n][4] row-major int32.  Constraint arrays list all PT pairs first, then
 *    all EE pairs.
 */
#ifndef BFAL_H
#define BFAL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BF_OK = 0,
  BF_WARN_PCG_MAXITER = 1,          /* PCG stopped at max_iter; p is the last iterate */
  BF_ERR_INVALID_ARG = -1,          /* null pointer, size, index out of range, non-finite value */
  BF_ERR_OOM = -2,                  /* device allocation failed */
  BF_ERR_HIP = -3,                  /* a HIP runtime call failed */
  BF_ERR_INVERTED_ELEMENT = -4,     /* det F(x_hat) <= 0 in some tet (Neo-Hookean is non-invertible) */
  BF_ERR_DEGENERATE_CONSTRAINT = -5,/* d_i(x) <= 0, repeated vertex, or (near-)parallel EE pair */
  BF_ERR_NOT_SPD = -6,              /* a diagonal block is not SPD, or PCG breakdown p^T H p <= 0 */
  BF_ERR_BUDGET = -7,               /* serving: a request's footprint exceeds the server's HBM budget */
  BF_ERR_STATE = -8                 /* call order: state or constraints missing */
} bf_status;

enum { BF_MEM_HOST = 0, BF_MEM_DEVICE = 1 };
enum { BF_PREC_FP32 = 0, BF_PREC_BF16_REFINE = 1 };

typedef struct bf_context bf_context;
typedef struct bf_problem bf_problem;

/* Tetrahedral mesh and material (Section 3; Neo-Hookean per tet). */
typedef struct {
  int32_t n_nodes, n_tets;
  const int32_t* tets;   /* [n_tets][4] vertex ids; positive orientation not required */
  const double* rest;    /* [n_nodes][3] rest positions */
  const double* E;       /* [n_tets] Young's modulus (Pa), > 0 */
  const double* nu;      /* [n_tets] Poisson ratio in (-1, 0.5) */
  const double* rho;     /* [n_tets] density (kg/m^3), > 0 */
  const uint8_t* fixed;  /* [n_nodes] 1 = Dirichlet node (Section 5.3); may be NULL */
  const int32_t* material; /* [n_tets] 0 Neo-Hookean, 1 stable Neo-Hookean, 2 corotated linear (Table 2);
                              NULL: all 0.  Neo-Hookean: mu/2 (I_C - 3) - mu ln J + lam/2 (ln J)^2; stable
                              Neo-Hookean (the rest-stable form of Smith, de Goes and Kim 2019): mu/2 (I_C - 3)
                              - mu (J - 1) + lam/2 (J - 1)^2; corotated linear (F = R S the polar
                              decomposition): mu |F - R|^2 + lam/2 (tr S - 3)^2.  Every tet must stay
                              uninverted (J > 0).  Host arrays are validated; on device arrays a value other
                              than 1 or 2 reads as 0. */
} bf_mesh_desc;

/* Active constraint set C = {(i, lambda_i, gamma_i)} (Algorithm 2 input). */
typedef struct {
  int32_t n_pt, n_ee;
  const int32_t* pt;     /* [n_pt][4]: p, t0, t1, t2 (four distinct vertices) */
  const int32_t* ee;     /* [n_ee][4]: a0, a1, b0, b1 (four distinct vertices) */
  const double* lambda;  /* [n_pt + n_ee] multiplier estimates, >= 0 */
  const double* gamma;   /* [n_pt + n_ee] decay factors in (0, 1]; NULL means all 1 */
  double kappa;          /* AL penalty stiffness (the paper's mu), > 0 */
  double delta;          /* surface separation offset (the paper's delta), >= 0 */
} bf_constraint_desc;

typedef struct {
  double tol;            /* stop at |r|_2 <= tol |b|_2 (unpreconditioned, FP64 norms); in BF16 mode the
                            relative tolerance of each inner solve against its own right-hand side */
  int32_t max_iter;      /* PCG iteration cap (BF_WARN_PCG_MAXITER when hit) */
  int32_t precision;     /* BF_PREC_FP32, or BF_PREC_BF16_REFINE: the scaled blocks are also stored
                            in BF16 (round to nearest even); each inner PCG runs on them with FP32
                            vectors and FP64 dot products; the outer loop keeps x in FP64 and forms
                            r = b - H x with the FP32 blocks in FP64 (iterative refinement) */
  double refine_tol;     /* BF16 mode: outer refinement stops at |b - H p|_2 <= refine_tol |b|_2 */
  int32_t poll_every;    /* host polls the device convergence flag every this many iterations */
  int32_t check_every;   /* the true residual norm is formed every this many iterations */
  int32_t time_spmv;     /* >0: time the SpMV launches of the first this-many PCG iterations
                            with HIP events (reported in bf_step_stats); 0: no per-kernel events */
  int32_t max_sweeps;    /* BF16 mode: at most this many inner solves (0 means 100) */
} bf_solve_opts;

typedef struct {
  int32_t pcg_iters;         /* inner PCG iterations (summed over sweeps in BF16 mode) */
  int32_t refine_sweeps;     /* inner solves of the refinement (BF16 mode), else 0 */
  double rel_residual;       /* final |b - H p|_2 / |b|_2 as tracked by the solver (FP64); in BF16
                                mode the FP64 residual of the FP32-stored system */
  double newton_inf_over_h;  /* |p|_inf / h (Section 6.1 residual-style stat), FP64 */
  double max_violation;      /* max_i max(0, -c_i(x_hat)), FP64 */
  int64_t nnzb;              /* stored upper 3x3 blocks, diagonal included */
  double ms_lin, ms_pattern, ms_assemble, ms_pcg;  /* device time per phase */
  int32_t spmv_timed;        /* SpMV launches timed (see bf_solve_opts.time_spmv) */
  double ms_spmv_avg;        /* their average duration (ms; events stamped around each dispatch) */
  double sweep_rel_residual[16]; /* BF16 mode: |b - H x_s|_2 / |b|_2 before inner solve s (FP64;
                                    entry 0 is 1), then after the last; unused entries 0 */
} bf_step_stats;

/* ---------------------------------------------------------------- context */

/* Open `device`.  `hip_stream` (a hipStream_t) is used for all work when
 * non-NULL; otherwise the context creates and owns a default-priority stream. */
bf_status bf_context_create(int32_t device, void* hip_stream, bf_context** out);
void bf_context_destroy(bf_context* ctx);
/* Message of the last failing call on this context ("" if none).  Owned by the
 * context, valid until its next call. */
const char* bf_last_error(const bf_context* ctx);

/* ---------------------------------------------------------------- problem */

/* Per-mesh setup: rest geometry (the constant row vectors A_a of Section 5.1),
 * Lame parameters, lumped mass (Section 3), the static elastic 3x3-block
 * pattern and its assembly order.  Copies the mesh.  Errors: INVALID_ARG for
 * bad sizes/indices/values or a degenerate rest tet. */
bf_status bf_problem_create(bf_context* ctx, const bf_mesh_desc* mesh, int32_t mem, bf_problem** out);
void bf_problem_destroy(bf_problem* pb);

/* x: intersection-free linearization point; x_hat: current iterate; x_tilde:
 * inertia target x^t + h v^t + h^2 M^{-1} f_ext (Section 3); dt = h > 0.
 * Each [n_nodes][3].  Copies them. */
bf_status bf_set_state(bf_problem* pb, const double* x, const double* x_hat, const double* x_tilde,
                       double dt, int32_t mem);

/* Copies and validates the active set.  Host memory is validated on the host;
 * device memory is validated by a kernel before any use. */
bf_status bf_set_constraints(bf_problem* pb, const bf_constraint_desc* cons, int32_t mem);

/* Semi-implicit friction (Appendix A; IPC's smoothed friction).  Captures the
 * friction set from the current constraints, multipliers, kappa and delta at
 * the current x (= x^t, the start of a time step): per contact its closest-point
 * weights w and normal n at x^t and coef = mu_f max(0, lambda - kappa (d(x^t) -
 * delta)), which is h^2 mu_f F^t with the previous step's normal force F^t.
 * Until the next call every Newton step, energy and subproblem adds, per
 * contact, coef f_0(|u|) with u the tangential part of sum_a w_a (x_hat_a -
 * x^t_a) and f_0 IPC's C^2 mollified norm with threshold eps_v h (h from
 * bf_set_state).  Later bf_set_constraints / bf_update_active_set calls leave
 * the friction set as captured.  mu_f = 0 clears it.  Requires bf_set_state
 * and bf_set_constraints (BF_ERR_STATE otherwise); mu_f >= 0 finite and, when
 * mu_f > 0, eps_v > 0 finite (BF_ERR_INVALID_ARG otherwise).  Allocates the
 * per-contact buffers on the device. */
bf_status bf_set_friction(bf_problem* pb, double mu_f, double eps_v);

/* One Newton step: constraint linearization at x, merged BSR pattern,
 * assembly of G and the SPD-projected H, block-Jacobi PCG for p = -H^{-1} G,
 * and the FP64 stats.  p_out is [n_nodes][3] doubles in `mem`.  stats may be
 * NULL.  Errors: INVERTED_ELEMENT, DEGENERATE_CONSTRAINT, NOT_SPD, STATE. */
bf_status bf_newton_step(bf_problem* pb, const bf_solve_opts* opts, double* p_out, int32_t mem,
                         bf_step_stats* stats);

/* ----------------------------------------------- introspection (parity) */
/* Valid after bf_newton_step.  All outputs are host memory. */

/* Assembled gradient G after DBC, [n_nodes][3]. */
bf_status bf_get_gradient(bf_problem* pb, double* g_out);
/* Number of stored upper blocks (diagonal included) of the last step. */
bf_status bf_get_nnzb(bf_problem* pb, int64_t* nnzb);
/* Upper BSR pattern: row_ptr [n_nodes+1], col [nnzb]; emap [n_tets][10] and
 * cmap [n_pt+n_ee][10] slots of the local vertex pairs (0,0),(0,1),(0,2),(0,3),
 * (1,1),(1,2),(1,3),(2,2),(2,3),(3,3) (the block is transposed when the first
 * vertex id is larger); diag [n_nodes] slot of (v,v).  Any pointer may be NULL. */
bf_status bf_get_pattern(bf_problem* pb, int32_t* row_ptr, int32_t* col, int32_t* emap, int32_t* cmap,
                         int32_t* diag);
/* Assembled (unscaled) blocks after DBC, [nnzb][3][3] row-major FP64 (the solver stores the
 * symmetrically scaled blocks rounded once to FP32). */
bf_status bf_get_blocks(bf_problem* pb, double* vals);

/* Device bytes a problem of this size holds (mesh, state, constraints,
 * pattern, blocks and solver vectors), for admission control. */
bf_status bf_footprint_bytes(int32_t n_nodes, int32_t n_tets, int32_t n_constraints, size_t* out);

/* ------------------------------------------------------------- subproblem */
/* The rest of SolveSubproblem (Algorithm 2; Section 4.2 "Alternating Primal
 * Solve" and "Constraint Decay") around bf_newton_step: from the x_hat of
 * bf_set_state, repeat Newton steps p = -H^{-1} G with a line search for the
 * first r in 1, 1/2, 1/4, ... (at most 30 halvings) with L(x_hat + r p) <
 * L(x_hat), x_hat += r p, until a full step (r = 1) is taken, no step
 * decreases L (r = 0) or max_newton steps were taken (a step whose PCG meets
 * negative curvature uses its iterate so far, as truncated Newton does, and
 * the call then returns BF_WARN_PCG_MAXITER); then update every
 * constraint from its slack s_i = max(0, c_i(x_hat) - lambda_i/kappa): s_i = 0
 * gives lambda_i -= kappa c_i and gamma_i = 1, s_i > 0 gives lambda_i = 0 and
 * gamma_i *= decay (the paper's Gamma, 0.9 in its experiments).  L is the
 * total energy of Section 4.2 with every slack at that minimizer, evaluated in
 * FP64; a state with an inverted tet has infinite energy. */
typedef struct {
  int32_t newton_iters;       /* Newton steps taken */
  int32_t pcg_iters;          /* PCG iterations summed over the steps */
  int32_t energy_evals;       /* energy evaluations (line searches included) */
  double energy_initial;      /* L(x_hat^0), FP64 */
  double energy_final;        /* L(x_hat) after the Newton loop (before the multiplier update) */
  double last_step;           /* r of the last step: 1 on the normal exit, 0 if no step decreased L */
  double max_violation;       /* max_i max(0, -c_i(x_hat)) at the multiplier update, FP64 */
  int32_t active;             /* constraints with s_i = 0 at the update */
  int32_t decayed;            /* constraints with s_i > 0 at the update */
  double ms_total;            /* device time of the call (steps, line searches) */
  int32_t truncated;          /* steps whose PCG met p^T H p <= 0 and used its iterate so far */
} bf_subproblem_stats;

/* Runs the loop above.  The problem keeps the final x_hat as its state and the
 * updated lambda and gamma as its constraint set (so calls chain as the outer
 * iterations of the augmented-Lagrangian method).  Outputs (any may be NULL)
 * in `mem`: x_hat_out [n_nodes][3], lambda_out and gamma_out [n_pt + n_ee].
 * Returns a warning when a Newton step's PCG hit max_iter. */
bf_status bf_solve_subproblem(bf_problem* pb, const bf_solve_opts* opts, int32_t max_newton, double decay,
                              double* x_hat_out, double* lambda_out, double* gamma_out, int32_t mem,
                              bf_subproblem_stats* stats);
/* L at the problem's current x_hat (FP64); *inverted = 1 (and L = inf) if a
 * tet is inverted.  Valid after a Newton step (it uses the linearization). */
bf_status bf_energy(bf_problem* pb, double* energy_out, int32_t* inverted);
/* bf_energy for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and result, with the per-workgroup partials, their sum and the
 * inversion flag in a static device array of the library (1 MiB per GPU, held
 * until the process ends) instead of a buffer of the problem; nothing is
 * allocated.  A problem needing more than that (8 bytes per 256 tets,
 * constraints and friction contacts, plus 64) gets BF_ERR_INVALID_ARG.  All
 * calls on one GPU share the array: calls that overlap on one GPU (several
 * threads or streams) race and must be serialized by the caller. */
bf_status bf_energy_noalloc(bf_problem* pb, double* energy_out, int32_t* inverted);

/* Conditioning-aware penalty (Section 5.2): *mu_out = C max_i (grad^2 E)_ii,
 * the largest scalar diagonal of the incremental potential's Hessian -- the
 * lumped mass plus h^2 times the SPD-projected elastic Hessian, the
 * matrix the Newton step assembles -- at x, the state the time step starts
 * from (bf_set_state's first argument).  The paper uses C = 0.1.  The caller
 * passes the result as kappa to bf_set_constraints.  Fixed nodes count: their
 * diagonals are kept by the moving-boundary elimination (Section 5.3).
 * Requires bf_set_state; C finite and > 0 (BF_ERR_INVALID_ARG otherwise);
 * BF_ERR_INVERTED_ELEMENT if a tet of x is inverted.  Computed from FP32 sums
 * of the element blocks.  Uses the step's staging buffer (no allocation after
 * the first Newton step or call). */
bf_status bf_mu_init(bf_problem* pb, double C, double* mu_out);

/* ------------------------------------------- collisions (Algorithms 1 and 3) */
/* The collision queries of the time step along the straight path from x (the
 * intersection-free state of bf_set_state) to a target x_hat: every surface
 * primitive pair -- point-triangle (a boundary vertex against a boundary
 * triangle of the tet mesh not containing it) and edge-edge (two boundary
 * edges without a common endpoint) -- whose swept boxes over both states come
 * within delta (bf_set_constraints) of each other on every axis is tested by
 * additive CCD (Li, Kaufman and Jiang 2021) in FP64 with separation ratio
 * sep: the pair "collides" when the conservative time at which its distance
 * would fall below sep times the initial one is below 1 (Section 5 uses a
 * linear BVH broad phase and ACCD narrow phase; the tree here is built per
 * call over FP32 boxes rounded outward, and every pair it reports is tested
 * again exactly).  A pair at distance 0 at x collides at t = 0; a pair still
 * stepping after 10^4 ACCD steps collides at the time reached.  The surface
 * is extracted from the tets at the first call.  x_hat: NULL for the
 * problem's current x_hat, else [N][3] FP64 in memory kind mem.  sep in
 * (0, 1); 0 selects 0.1.  Requires bf_set_state and bf_set_constraints. */
typedef struct {
  int64_t candidates_pt, candidates_ee; /* pairs passing the exact swept-box test */
  int32_t colliding_pt, colliding_ee;   /* of those, pairs whose collision time is below 1 */
  int32_t new_pt, new_ee;               /* colliding pairs not in the active set, near-parallel edge pairs
                                           excluded (update only) */
  int32_t added_pt, added_ee;           /* new pairs kept by the earliest-time filter (update only) */
  int32_t removed;                      /* constraints dropped for gamma < 0.01 (update only) */
  int32_t n_pt, n_ee;                   /* size of the active set after the call */
  double alpha_ccd;                     /* smallest collision time (1 if none) */
  double alpha_inversion;               /* smallest inversion bound over the tets (1 if none) */
  double ms_tree, ms_query, ms_update;  /* device time: BVH builds, queries with ACCD, set rebuild */
} bf_ccd_stats;

/* UpdateActiveSet (Algorithm 3): of the colliding pairs not already in the
 * active set (compared by vertex sets), every vertex takes the earliest
 * collision time T_v of the new pairs it belongs to, and a new pair is kept
 * when its time equals T_v for one of its vertices (up to the times' FP64
 * rounding: T_i <= T_v (1 + 1e-9)); it enters with lambda = 0,
 * gamma = 1.  An edge pair (near-)parallel at x (|e_a x e_b|^2 < 1e-8
 * |e_a|^2 |e_b|^2, where the distance gradient is not unique and a Newton
 * step would reject the constraint) does not enter the set and is not
 * counted in new_ee; it still limits bf_max_step_size.  Constraints whose
 * gamma fell below 0.01 are removed.  The new
 * active set, device-resident, is: the surviving PT constraints in their
 * order, the new PT pairs (p, t0 < t1 < t2) ordered by (p, triangle), the
 * surviving EE constraints, the new EE pairs (a0 < a1, b0 < b1, edge a before
 * edge b) ordered by (edge a, edge b).  kappa and delta stay.  bf_energy then
 * needs a new Newton step. */
bf_status bf_update_active_set(bf_problem* pb, const double* x_hat, int32_t mem, double sep, bf_ccd_stats* stats);

/* MaxStepSize (Algorithm 1): *alpha = min(1, the smallest collision time of
 * the colliding pairs, the smallest inversion bound), where a tet's inversion
 * bound is the first t in (0, 1] with det D_s(t) = sep det D_s(0) along the
 * path (the Neo-Hookean energy is non-invertible), found by bisection between
 * the roots of the cubic's derivative. */
bf_status bf_max_step_size(bf_problem* pb, const double* x_hat, int32_t mem, double sep, double* alpha,
                           bf_ccd_stats* stats);

/* Introspection for the parity tests: the colliding pairs of the last
 * collision call (bf_update_active_set or bf_max_step_size), in no particular
 * order -- PT rows (p, t0 < t1 < t2) and EE rows (a0 < a1, b0 < b1, edge a
 * before edge b) with their collision times, host memory, sized by the
 * call's colliding_pt / colliding_ee; NULL skips an array. */
bf_status bf_get_collisions(bf_problem* pb, int32_t* pt, double* pt_toc, int32_t* ee, double* ee_toc);

/* The active set: counts, then the arrays (PT rows [n_pt][4], EE rows
 * [n_ee][4], lambda and gamma [n_pt + n_ee], PT first) in memory kind mem;
 * NULL skips an array. */
bf_status bf_get_constraint_counts(bf_problem* pb, int32_t* n_pt, int32_t* n_ee);
bf_status bf_get_constraints(bf_problem* pb, int32_t* pt, int32_t* ee, double* lambda, double* gamma, int32_t mem);

/* ---------------------------------------------------------- time step */
/* One time step (Algorithm 1, Section 4.1) from the problem's state: x = x^t
 * (intersection free), x_hat = x_hat^[0] (x^t with the moving-boundary nodes
 * at their targets, Section 5.3), x_tilde and h from bf_set_state, the active
 * set of bf_set_constraints (or of the previous step).  Repeats
 *   x_hat <- SolveSubproblem (bf_solve_subproblem: Newton steps with the line
 *            search until a full step, then the multiplier / decay update),
 *   C     <- UpdateActiveSet along x -> the subproblem's input x_hat
 *            (bf_update_active_set),
 *   alpha <- MaxStepSize along x -> the new x_hat (bf_max_step_size),
 *   x     <- (1 - alpha) x + alpha x_hat,
 *   beta  <- (1 - alpha) beta once k + 1 >= k_min,
 * while beta > eps (Section 6: eps = 1e-3, k_min = 2).  Section 5.2: with
 * mu_init_c > 0 the penalty starts at mu_init_c max_i (grad^2 E)_ii
 * (bf_mu_init; the paper uses 0.1), and whenever alpha stays below 1e-4 for
 * 50 consecutive iterations kappa doubles and delta halves.  Friction
 * (Appendix A): the step first calls bf_set_friction(mu_f, eps_v), so the
 * friction set comes from the incoming active set and multipliers at x^t and
 * holds for the whole step; mu_f = 0 steps without friction (and clears a
 * set captured earlier).  The paper uses k_min = 6 with friction.  On return the
 * problem holds x^{t+1}, the last x_hat and the active set with its
 * multipliers; x_out and v_out = (x^{t+1} - x^t) / h ([N][3] FP64, kind mem,
 * nullable) receive the state.  Returns BF_WARN_PCG_MAXITER when max_outer
 * ends the loop (or a Newton step's PCG warned), errors of the calls above
 * otherwise. */
typedef struct {
  bf_solve_opts solve;  /* the Newton steps' linear solves */
  int32_t k_min;        /* K_min >= 1 */
  double eps;           /* termination threshold on beta, in (0, 1) */
  int32_t max_outer;    /* cap on the iterations, >= 1 */
  int32_t max_newton;   /* Newton steps per subproblem, >= 1 */
  double decay;         /* Gamma of the constraint decay, in (0, 1] */
  double sep;           /* ACCD separation ratio (0 selects 0.1) */
  double mu_init_c;     /* > 0: start from mu_init_c max_i (grad^2 E)_ii; 0 keeps kappa */
  double mu_f;          /* friction coefficient (0: no friction) */
  double eps_v;         /* friction smoothing: f_0 is |u| beyond eps_v h (used when mu_f > 0) */
} bf_time_step_opts;

typedef struct {
  int32_t outer_iters, newton_iters, pcg_iters, truncated;
  double beta;          /* final cumulative weight of x^t */
  double alpha_min, alpha_last;
  int32_t n_pt, n_ee;   /* active set at the end */
  int32_t mu_doublings;
  double kappa, delta;  /* at the end */
  double ms_subproblem, ms_ccd, ms_total;   /* device time of the subproblems and collision calls; wall time */
} bf_time_step_stats;

bf_status bf_time_step(bf_problem* pb, const bf_time_step_opts* o, double* x_out, double* v_out, int32_t mem,
                       bf_time_step_stats* stats);

/* ---------------------------------------------------------------- serving */
/* A server solves independent Newton-step requests (each: a mesh, its state
 * and its active constraint set; the same operation as bf_newton_step, FP32
 * mode) with continuous batching on one device.  Two threads of the library
 * work in the background: admission threads take submitted requests in
 * arrival order and admits the head of the queue when its footprint
 * (bf_footprint_bytes) fits beside the admitted ones in hbm_budget and fewer
 * than max_active are admitted, then assembles it on its own stream; a batch
 * thread runs the PCG of all admitted requests in shared launches (a
 * block-diagonal system with per-request scalars, iters_per_round iterations
 * between scheduling points), retires finished requests and frees their
 * budget.  Requests arriving while others are on the GPU join the batch as
 * slots and memory free up; several admission workers assemble arriving
 * requests concurrently.  max_active = 1 serves one request at a time.
 * Threads: submit, poll, result and stats may be called from any one thread;
 * the server uses its own streams, so the calling thread's context is free. */
typedef struct bf_server bf_server;
typedef struct {
  size_t hbm_budget;         /* device bytes the admitted requests may hold (footprint estimates), > 0 */
  int32_t max_active;        /* at most this many admitted requests, >= 1 */
  int32_t iters_per_round;   /* batched PCG iterations between scheduling points, >= 1 */
  int32_t admit_threads;     /* admission workers (each assembles on its own stream); 0 means 3, which with
                                the batch stream keeps to the 4 hardware queues a process gets */
} bf_server_opts;
typedef struct {
  double t_submit, t_admit, t_done;  /* seconds on bf_clock_now()'s clock */
} bf_request_times;

/* A monotonic clock (seconds) shared with the request time stamps. */
double bf_clock_now(void);
bf_status bf_server_create(int32_t device, const bf_server_opts* opts, bf_server** out);
/* Copies the request (host memory only) and queues it; returns at once.
 * req_id must not be queued or finished-but-untaken already.  The arrays are
 * checked here as the single-problem calls check them (bf_check_mesh,
 * bf_check_state, bf_check_constraints, bf_check_solve_opts of bfal_host.h),
 * and a failing check is returned at once; opts->precision must be
 * BF_PREC_FP32.  Errors found on the device (an inverted element, a degenerate
 * constraint) and BF_ERR_BUDGET are reported through the request's status
 * (bf_server_result). */
bf_status bf_server_submit(bf_server* srv, int64_t req_id, const bf_mesh_desc* mesh, const double* x,
                           const double* x_hat, const double* x_tilde, double dt,
                           const bf_constraint_desc* cons, const bf_solve_opts* opts);
/* Non-blocking: writes up to cap ids of requests finished since the last poll. */
bf_status bf_server_poll(bf_server* srv, int64_t* done_ids, int32_t cap, int32_t* n_done);
/* Takes a finished request's result: p_out [n_nodes][3] host doubles, stats,
 * times and its status (a bf_status: BF_OK, a warning or an error such as
 * BF_ERR_BUDGET when its footprint exceeds the whole budget).  Any output may
 * be NULL.
 * BF_ERR_STATE if the id is not finished. */
bf_status bf_server_result(bf_server* srv, int64_t req_id, double* p_out, bf_step_stats* stats,
                           bf_request_times* times, int32_t* req_status);
/* Queue length, admitted requests and their footprint sum. */
bf_status bf_server_stats(bf_server* srv, int32_t* n_pending, int32_t* n_active, size_t* used_bytes);
/* Stops the threads (requests still queued or running are dropped) and frees everything. */
void bf_server_destroy(bf_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* BFAL_H */
