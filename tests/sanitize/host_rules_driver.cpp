// Drives every host rule of libbfal (include/bfal_host.h) through valid and
// invalid inputs; built together with host_rules.cpp under AddressSanitizer
// and UndefinedBehaviorSanitizer by tests/test_host_sanitizers_cpu.py.
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/bfal_host.h"

static int failures = 0;
#define EXPECT(cond)                                                  \
  do {                                                                \
    if (!(cond)) {                                                    \
      std::fprintf(stderr, "%s:%d: %s\n", __FILE__, __LINE__, #cond); \
      ++failures;                                                     \
    }                                                                 \
  } while (0)

int main() {
  // one tet, valid
  const int32_t tets[4] = {0, 1, 2, 3};
  const double rest[12] = {0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0, 1};
  const double E[1] = {1e5}, nu[1] = {0.3}, rho[1] = {1e3};
  char msg[8];   // short on purpose: messages are truncated, never overrun
  bf_mesh_desc m{4, 1, tets, rest, E, nu, rho, nullptr, nullptr};
  EXPECT(bf_check_mesh(&m, msg, sizeof msg) == BF_OK);
  EXPECT(bf_check_mesh(nullptr, msg, sizeof msg) == BF_ERR_INVALID_ARG);
  EXPECT(std::strlen(msg) == sizeof msg - 1);
  EXPECT(bf_check_mesh(&m, nullptr, 0) == BF_OK);
  bf_mesh_desc big = m;
  big.n_tets = 1 << 30;   // rejected by size before any array is read
  EXPECT(bf_check_mesh(&big, msg, sizeof msg) == BF_ERR_INVALID_ARG);
  const int32_t bad_tets[4] = {0, 1, 2, 4};
  bf_mesh_desc bm = m;
  bm.tets = bad_tets;
  EXPECT(bf_check_mesh(&bm, msg, 0) == BF_ERR_INVALID_ARG);
  const int32_t mat[1] = {-1};
  bf_mesh_desc mm = m;
  mm.material = mat;
  EXPECT(bf_check_mesh(&mm, msg, sizeof msg) == BF_ERR_INVALID_ARG);

  // state
  std::vector<double> x(12, 0.0);
  EXPECT(bf_check_state(4, x.data(), x.data(), x.data(), 0.01, msg, sizeof msg) == BF_OK);
  EXPECT(bf_check_state(4, x.data(), nullptr, x.data(), 0.01, msg, sizeof msg) == BF_ERR_INVALID_ARG);
  EXPECT(bf_check_state(4, x.data(), x.data(), x.data(), -1.0, msg, sizeof msg) == BF_ERR_INVALID_ARG);
  EXPECT(bf_check_state(0, x.data(), x.data(), x.data(), 0.01, msg, sizeof msg) == BF_ERR_INVALID_ARG);

  // constraints
  const int32_t pt[4] = {0, 1, 2, 3}, ee[4] = {0, 1, 2, 2};
  const double lam[2] = {1.0, 2.0}, gam[2] = {1.0, 0.5};
  bf_constraint_desc cd{1, 0, pt, nullptr, lam, gam, 1e4, 1e-3};
  EXPECT(bf_check_constraints(4, &cd, msg, sizeof msg) == BF_OK);
  bf_constraint_desc ce{1, 1, pt, ee, lam, gam, 1e4, 1e-3};
  EXPECT(bf_check_constraints(4, &ce, msg, sizeof msg) == BF_ERR_DEGENERATE_CONSTRAINT);
  bf_constraint_desc cn{1, 1, pt, nullptr, lam, gam, 1e4, 1e-3};
  EXPECT(bf_check_constraints(4, &cn, msg, sizeof msg) == BF_ERR_INVALID_ARG);
  bf_constraint_desc ch{1 << 29, 1 << 29, pt, ee, lam, gam, 1e4, 1e-3};   // count overflow caught before reads
  EXPECT(bf_check_constraints(4, &ch, msg, sizeof msg) == BF_ERR_INVALID_ARG);
  EXPECT(bf_check_constraints(4, nullptr, msg, sizeof msg) == BF_ERR_INVALID_ARG);

  // solve options
  bf_solve_opts o{1e-5, 100, BF_PREC_FP32, 1e-6, 16, 1, 0, 0};
  EXPECT(bf_check_solve_opts(&o, msg, sizeof msg) == BF_OK);
  o.precision = 9;
  EXPECT(bf_check_solve_opts(&o, msg, sizeof msg) == BF_ERR_INVALID_ARG);
  EXPECT(bf_check_solve_opts(nullptr, msg, sizeof msg) == BF_ERR_INVALID_ARG);

  // stall rule
  bf_stall_rule r{1e-4, 3, 0};
  double kappa = 1.0, delta = 1.0;
  EXPECT(bf_stall_step(&r, 1e-6, &kappa, &delta) == 0);
  EXPECT(bf_stall_step(&r, 1e-6, &kappa, &delta) == 0);
  EXPECT(bf_stall_step(&r, 1e-6, &kappa, &delta) == 1);
  EXPECT(kappa == 2.0 && delta == 0.5 && r.count == 0);
  EXPECT(bf_stall_step(nullptr, 0.0, &kappa, &delta) == -1);
  bf_stall_rule rz{1e-4, 0, 0};
  EXPECT(bf_stall_step(&rz, 0.0, &kappa, &delta) == -1);

  // admission: a long random-looking sequence, freed in a scrambled order
  bf_admission* a = nullptr;
  EXPECT(bf_admission_create(0, 4, &a) == BF_ERR_INVALID_ARG);
  EXPECT(bf_admission_create(1000, 4, &a) == BF_OK);
  std::vector<int32_t> slots;
  uint64_t seed = 12345;
  for (int i = 0; i < 5000; ++i) {
    seed = seed * 6364136223846793005ULL + 1442695040888963407ULL;
    const uint64_t f = 1 + (seed >> 33) % 1200;   // some never fit
    EXPECT(bf_admission_push(a, i, f) == BF_OK);
    int64_t id;
    int32_t s;
    int32_t d;
    while ((d = bf_admission_next(a, &id, &s)) != 0) {
      if (d == 1) slots.push_back(s);
    }
    EXPECT(bf_admission_used(a) <= 1000);
    if (slots.size() >= 3 || (seed & 1)) {
      while (!slots.empty()) {
        const size_t k = (seed >> 7) % slots.size();
        // the policy checks the footprint released against the one admitted
        // into the slot: try sizes until it accepts (every wrong one is refused)
        uint64_t want = 0;
        for (uint64_t g = 1; g <= 1200; ++g)
          if (bf_admission_release(a, slots[k], g) == BF_OK) {
            want = g;
            break;
          }
        EXPECT(want > 0);
        slots.erase(slots.begin() + k);
      }
    }
  }
  EXPECT(bf_admission_active(a) >= 0 && bf_admission_waiting(a) >= 0);
  bf_admission_destroy(a);
  bf_admission_destroy(nullptr);
  // slice plan: random widths, every slice listed once, lists increasing
  for (int trial = 0; trial < 20; ++trial) {
    seed = seed * 6364136223846793005ULL + 1442695040888963407ULL;
    const int32_t ns = 1 + (int32_t)((seed >> 33) % 3000), nparts = 8 * (1 + (int32_t)((seed >> 20) % 64));
    std::vector<int32_t> su(ns + 1, 0), sl(ns + 1, 0), ptr(nparts + 1), ws(ns);
    for (int32_t s = 0; s < ns; ++s) {
      seed = seed * 6364136223846793005ULL + 1442695040888963407ULL;
      su[s + 1] = su[s] + 64 * (int32_t)((seed >> 40) % 20);
      sl[s + 1] = sl[s] + 64 * (int32_t)((seed >> 50) % 20);
    }
    EXPECT(bf_slice_plan(ns, su.data(), sl.data(), 2, nparts, ptr.data(), ws.data()) == BF_OK);
    std::vector<int> seen(ns, 0);
    EXPECT(ptr[0] == 0 && ptr[nparts] == ns);
    for (int32_t p = 0; p < nparts; ++p)
      for (int32_t j = ptr[p]; j < ptr[p + 1]; ++j) {
        EXPECT(ws[j] >= 0 && ws[j] < ns);
        if (ws[j] >= 0 && ws[j] < ns) ++seen[ws[j]];
        if (j > ptr[p]) EXPECT(ws[j] > ws[j - 1]);
      }
    for (int32_t s = 0; s < ns; ++s) EXPECT(seen[s] == 1);
  }
  {
    std::vector<int32_t> su = {0, 64, 100}, sl = {0, 64, 128}, ptr(9), ws(2);
    EXPECT(bf_slice_plan(2, su.data(), sl.data(), 2, 8, ptr.data(), ws.data()) == BF_ERR_INVALID_ARG);
    EXPECT(bf_slice_plan(2, sl.data(), sl.data(), 2, 12, ptr.data(), ws.data()) == BF_ERR_INVALID_ARG);
    EXPECT(bf_slice_plan(2, sl.data(), sl.data(), 2, 8, nullptr, ws.data()) == BF_ERR_INVALID_ARG);
  }
  if (failures) return 1;
  std::printf("host rules: all checks passed\n");
  return 0;
}
