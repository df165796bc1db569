// One time step (Algorithm 1) on the device state of a problem: alternate
// SolveSubproblem (Algorithm 2), UpdateActiveSet (Algorithm 3) and
// MaxStepSize, moving the intersection-free state x^[k] toward each new
// target, until the cumulative weight beta of the starting state falls below
// eps.  Host orchestration only: every step runs in the kernels behind the
// entry points it calls.
#include <algorithm>
#include <chrono>

#include "problem.h"

using namespace bfal;

extern "C" {

bf_status bf_time_step(bf_problem* pb, const bf_time_step_opts* o, double* x_out, double* v_out, int32_t mem,
                       bf_time_step_stats* stats) {
  if (!pb) return BF_ERR_INVALID_ARG;
  bf_context* c = pb->ctx;
  if (!o) return fail(c, BF_ERR_INVALID_ARG, "opts is NULL");
  if (o->k_min < 1) return fail(c, BF_ERR_INVALID_ARG, "k_min must be >= 1");
  if (!(o->eps > 0.0 && o->eps < 1.0)) return fail(c, BF_ERR_INVALID_ARG, "eps must lie in (0, 1)");
  if (o->max_outer < 1 || o->max_newton < 1) return fail(c, BF_ERR_INVALID_ARG, "max_outer and max_newton >= 1");
  if (!(o->decay > 0.0 && o->decay <= 1.0)) return fail(c, BF_ERR_INVALID_ARG, "decay must lie in (0, 1]");
  if (!(o->mu_init_c >= 0.0)) return fail(c, BF_ERR_INVALID_ARG, "mu_init_c must be >= 0");
  if (mem != BF_MEM_HOST && mem != BF_MEM_DEVICE) return fail(c, BF_ERR_INVALID_ARG, "bad mem kind");
  if (!pb->has_state) return fail(c, BF_ERR_STATE, "bf_set_state must be called first");
  if (pb->cap_nnzb == 0) return fail(c, BF_ERR_STATE, "bf_set_constraints must be called first");
  HIPCHK(c, hipSetDevice(c->device));
  hipStream_t s = c->stream;
  const auto t_start = std::chrono::steady_clock::now();
  const long long n3 = 3LL * pb->N;
  ALLOC(c, pb->xstart, 8 * n3);
  ALLOC(c, pb->xprev, 8 * n3);
  HIPCHK(c, hipMemcpyAsync(pb->xstart.p, pb->x.p, 8 * n3, hipMemcpyDeviceToDevice, s));
  bf_time_step_stats out{};
  bf_status warn = BF_OK;
  {
    // the friction set of this step, from the incoming contacts at x^t (Appendix A)
    bf_status st = bf_set_friction(pb, o->mu_f, o->eps_v);
    if (st != BF_OK) return st;
  }
  if (o->mu_init_c > 0.0) {
    double mu = 0.0;
    bf_status st = bf_mu_init(pb, o->mu_init_c, &mu);
    if (st != BF_OK) return st;
    pb->kappa = mu;
  }
  double beta = 1.0;
  int k = 0;
  bf_stall_rule stall{1e-4, 50, 0};   // Section 5.2
  out.alpha_min = 1.0;
  while (beta > o->eps && k < o->max_outer) {
    HIPCHK(c, hipMemcpyAsync(pb->xprev.p, pb->xh.p, 8 * n3, hipMemcpyDeviceToDevice, s));
    bf_subproblem_stats sst{};
    bf_status st = bf_solve_subproblem(pb, &o->solve, o->max_newton, o->decay, nullptr, nullptr, nullptr,
                                       BF_MEM_DEVICE, &sst);
    if (st < 0) return st;
    if (st > 0) warn = st;
    out.newton_iters += sst.newton_iters;
    out.pcg_iters += sst.pcg_iters;
    out.truncated += sst.truncated;
    out.ms_subproblem += sst.ms_total;
    bf_ccd_stats cst{};
    st = bf_update_active_set(pb, pb->xprev.as<double>(), BF_MEM_DEVICE, o->sep, &cst);
    if (st != BF_OK) return st;
    double alpha = 1.0;
    bf_ccd_stats mst{};
    st = bf_max_step_size(pb, nullptr, BF_MEM_DEVICE, o->sep, &alpha, &mst);
    if (st != BF_OK) return st;
    out.ms_ccd += cst.ms_tree + cst.ms_query + cst.ms_update + mst.ms_tree + mst.ms_query;
    launch_blend((int)n3, pb->x.as<double>(), pb->xh.as<double>(), alpha, s);
    if (k + 1 >= o->k_min) beta *= 1.0 - alpha;
    out.alpha_min = std::min(out.alpha_min, alpha);
    out.alpha_last = alpha;
    // Section 5.2: double the penalty and halve the offset when the step
    // stays below 1e-4 for 50 consecutive iterations
    if (bf_stall_step(&stall, alpha, &pb->kappa, &pb->delta) == 1) ++out.mu_doublings;
    ++k;
  }
  HIPCHK(c, hipStreamSynchronize(s));
  if (x_out) HIPCHK(c, hipMemcpyAsync(x_out, pb->x.p, 8 * n3, kind_out(mem), s));
  if (v_out) {
    ALLOC(c, pb->vout, 8 * n3);
    launch_velocity((int)n3, pb->x.as<double>(), pb->xstart.as<double>(), 1.0 / pb->dt, pb->vout.as<double>(), s);
    HIPCHK(c, hipMemcpyAsync(v_out, pb->vout.p, 8 * n3, kind_out(mem), s));
  }
  HIPCHK(c, hipStreamSynchronize(s));
  out.outer_iters = k;
  out.beta = beta;
  out.n_pt = pb->n_pt;
  out.n_ee = pb->n_ee;
  out.kappa = pb->kappa;
  out.delta = pb->delta;
  out.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  if (stats) *stats = out;
  c->err.clear();
  if (beta > o->eps) {
    c->err = "time step reached max_outer before beta <= eps";
    return BF_WARN_PCG_MAXITER;
  }
  return warn;
}

}  // extern "C"
