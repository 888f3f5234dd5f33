// Host-side exercise of the C ABI for the sanitizer build (AddressSanitizer
// and UndefinedBehaviorSanitizer on the plan and driver code): problem
// validation and rejection, the enumeration of the index set, coefficient
// tables, launch shapes and scratch sizing of plan creation for every
// operator (up to the first device allocation on a host without a GPU; to
// the end and through destroy where a GPU is present), the shape entry
// points on a live plan, and every entry point with NULL arguments.
// Prints one line per check and exits non-zero on the first failure.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "ctm.h"

static int failures = 0;
#define CHECK(cond, ...)                      \
  do {                                        \
    if (!(cond)) {                            \
      std::printf("FAIL: " __VA_ARGS__);      \
      std::printf("\n");                      \
      ++failures;                             \
    }                                         \
  } while (0)

struct Tables {
  std::vector<double> w, f;
};

// u0 = prod_i sin(pi (x_i - lo_i) / (hi_i - lo_i)) tabulated on the finest
// 1-D nodes (a smooth start for every operator; the lattice gets a delta)
static void fill(ctm_problem& p, Tables& t, bool lattice) {
  const int F = (1 << p.level_n) + 1;
  t.w.assign(1, 1.0);
  t.f.assign((size_t)p.d * F, 0.0);
  for (int i = 0; i < p.d; ++i)
    for (int J = 0; J < F; ++J)
      t.f[(size_t)i * F + J] = lattice ? (J == 0 ? 1.0 : 0.0) : std::sin(M_PI * J / (F - 1));
  p.ic_terms = 1;
  p.ic_weight = t.w.data();
  p.ic_factor = t.f.data();
}

static ctm_problem base(int d, int n, ctm_op_kind op) {
  ctm_problem p;
  ctm_problem_defaults(&p);
  p.d = d;
  p.level_n = n;
  p.op = op;
  for (int i = 0; i < d; ++i) {
    p.lo[i] = (op == CTM_OP_CME) ? 0.0 : -1.0;
    p.hi[i] = (op == CTM_OP_CME) ? std::ldexp(1.0, n) : 1.0;
    p.theta[i] = 1.0 + 0.1 * i;
    p.k[i] = 10.0;
    p.gamma[i] = 1.0;
  }
  p.sigma = 1.0;
  p.amp = 0.5;
  p.nsteps = 64;
  p.t1 = 0.1;
  if (op == CTM_OP_DRIFT)
    for (int i = 0; i < d; ++i) {
      p.diffusion[i] = 0.2;
      p.drift[i * d + i] = -1.0;
      if (i + 1 < d) p.drift[i * d + i + 1] = 0.5;
    }
  return p;
}

// Create; if a device is present, walk the queries and the shape entry
// points, then destroy. On a host without one, creation must fail cleanly.
static void create_cycle(ctm_problem p, const char* what) {
  Tables t;
  fill(p, t, p.op == CTM_OP_CME);
  ctm_plan* plan = nullptr;
  const ctm_status st = ctm_plan_create(&p, &plan);
  if (st != CTM_OK) {
    CHECK(plan == nullptr, "%s: failed creation left a plan", what);
    CHECK(st == CTM_ERR_HIP || st == CTM_ERR_NOMEM, "%s: creation status %d (%s)", what, (int)st,
          ctm_last_error());
    std::printf("ok   %-44s create -> %s (%s)\n", what, ctm_status_string(st), ctm_last_error());
    return;
  }
  int G = 0;
  long long len = 0;
  size_t ws = 0;
  CHECK(ctm_plan_grids(plan, &G) == CTM_OK && G > 0, "%s: grids", what);
  CHECK(ctm_plan_state_len(plan, &len) == CTM_OK && len > 0, "%s: state_len", what);
  CHECK(ctm_plan_workspace_bytes(plan, &ws) == CTM_OK, "%s: workspace", what);
  long long sum = 0;
  for (int g = 0; g < G; ++g) {
    int lev[CTM_MAXD];
    double coef = 0;
    long long off = -1, np = 0;
    CHECK(ctm_plan_grid_info(plan, g, lev, &coef, &off, &np) == CTM_OK, "%s: grid_info", what);
    CHECK(off == sum, "%s: grid %d offset", what, g);
    sum += np;
    int w = 0, k = 0;
    CHECK(ctm_plan_grid_shape(plan, g, &w, &k) == CTM_OK, "%s: grid_shape", what);
    if (k) ctm_plan_set_grid_shape(plan, g, w, k == 4 ? 8 : 4);  // may be refused
    ctm_plan_set_grid_shape(plan, g, 3, 4);                      // no such shape
  }
  CHECK(sum == len, "%s: offsets sum to the state length", what);
  CHECK(ctm_plan_grid_info(plan, G, nullptr, nullptr, nullptr, nullptr) == CTM_ERR_INVALID,
        "%s: grid index out of range accepted", what);
  CHECK(ctm_plan_set_wide(plan, -1) == CTM_ERR_INVALID, "%s: negative wide count", what);
  CHECK(ctm_plan_set_wide(plan, 1 << 30) == CTM_OK, "%s: large wide count", what);
  ctm_plan_destroy(plan);
  std::printf("ok   %-44s create -> ok, %d grids, %lld unknowns\n", what, G, len);
}

int main() {
  // every entry point with NULL arguments
  CHECK(ctm_problem_defaults(nullptr) == CTM_ERR_INVALID, "defaults(NULL)");
  CHECK(ctm_plan_create(nullptr, nullptr) == CTM_ERR_INVALID, "create(NULL, NULL)");
  ctm_plan* none = nullptr;
  CHECK(ctm_plan_create(nullptr, &none) == CTM_ERR_INVALID && none == nullptr, "create(NULL)");
  ctm_plan_destroy(nullptr);
  int G;
  long long ll;
  size_t sz;
  ctm_stats stats;
  CHECK(ctm_plan_grids(nullptr, &G) == CTM_ERR_INVALID, "grids(NULL)");
  CHECK(ctm_plan_state_len(nullptr, &ll) == CTM_ERR_INVALID, "state_len(NULL)");
  CHECK(ctm_plan_workspace_bytes(nullptr, &sz) == CTM_ERR_INVALID, "workspace(NULL)");
  CHECK(ctm_get_stats(nullptr, &stats) == CTM_ERR_INVALID, "get_stats(NULL)");
  CHECK(ctm_solve(nullptr, nullptr, 0, nullptr, nullptr, nullptr) == CTM_ERR_INVALID, "solve(NULL)");
  CHECK(ctm_gather(nullptr, nullptr, nullptr, 0, nullptr, nullptr) == CTM_ERR_INVALID, "gather(NULL)");
  CHECK(ctm_set_timing(nullptr, 1) == CTM_ERR_INVALID, "set_timing(NULL)");
  CHECK(ctm_plan_set_wide(nullptr, 1) == CTM_ERR_INVALID, "set_wide(NULL)");
  CHECK(ctm_plan_set_schedule(nullptr, 1) == CTM_ERR_INVALID, "set_schedule(NULL)");
  CHECK(ctm_precond_apply(nullptr, 0, nullptr, nullptr, nullptr) == CTM_ERR_INVALID,
        "precond_apply(NULL)");
  CHECK(std::strlen(ctm_status_string((ctm_status)99)) > 0, "status string of an unknown code");
  std::printf("ok   NULL arguments\n");

  // rejected problems: validation runs before any allocation
  struct Bad {
    const char* what;
    void (*mutate)(ctm_problem&);
  } bad[] = {
      {"d = 0", [](ctm_problem& p) { p.d = 0; }},
      {"d = 9", [](ctm_problem& p) { p.d = 9; }},
      {"level_min = 0", [](ctm_problem& p) { p.level_min = 0; }},
      {"n below d L0", [](ctm_problem& p) { p.level_min = 4; }},
      {"n + d - 1 > 30", [](ctm_problem& p) { p.level_n = 30; }},
      {"empty box", [](ctm_problem& p) { p.hi[1] = p.lo[1]; }},
      {"t1 <= t0", [](ctm_problem& p) { p.t1 = p.t0; }},
      {"nsteps = 0", [](ctm_problem& p) { p.nsteps = 0; }},
      {"nrecomb does not divide", [](ctm_problem& p) { p.nrecomb = 3; }},
      {"cf = 1", [](ctm_problem& p) { p.mgrit_cf = 1; }},
      {"cf^(L-1) does not divide", [](ctm_problem& p) { p.mgrit_cf = 3; }},
      {"mgrit_tol = 0", [](ctm_problem& p) { p.mgrit_tol = 0; }},
      {"krylov_tol NaN", [](ctm_problem& p) { p.krylov_tol = NAN; }},
      {"krylov_maxit = 0", [](ctm_problem& p) { p.krylov_maxit = 0; }},
      {"unknown operator", [](ctm_problem& p) { int v = 17; std::memcpy(&p.op, &v, sizeof v); }},
      {"unknown precision", [](ctm_problem& p) { int v = 5; std::memcpy(&p.prec, &v, sizeof v); }},
      {"unknown Krylov method", [](ctm_problem& p) { int v = 9; std::memcpy(&p.krylov, &v, sizeof v); }},
      {"unknown relaxation", [](ctm_problem& p) { int v = -1; std::memcpy(&p.relax, &v, sizeof v); }},
      {"unknown manufactured problem",
       [](ctm_problem& p) { int v = 4; std::memcpy(&p.manufactured, &v, sizeof v); }},
      {"coarse_tol = 1", [](ctm_problem& p) { p.coarse_tol = 1.0; }},
      {"no initial value", [](ctm_problem& p) { p.ic_terms = 0; }},
      {"17 initial terms", [](ctm_problem& p) { p.ic_terms = 17; }},
      {"residual mode on one level", [](ctm_problem& p) { p.residual_mode = 1; p.mgrit_levels = 1; }},
      {"mixed with refine_tol 0", [](ctm_problem& p) { p.prec = CTM_PREC_MIXED; p.refine_tol = 0; }},
      {"unknown preconditioner", [](ctm_problem& p) { int v = 3; std::memcpy(&p.precond, &v, sizeof v); }},
      {"Schwarz S = 1", [](ctm_problem& p) { p.precond = CTM_PRECOND_SCHWARZ; p.schwarz_s = 1; }},
      {"Schwarz S = 7", [](ctm_problem& p) { p.precond = CTM_PRECOND_SCHWARZ; p.schwarz_s = 7; }},
  };
  for (const Bad& b : bad) {
    ctm_problem p = base(2, 5, CTM_OP_HEAT);
    Tables t;
    fill(p, t, false);
    b.mutate(p);
    // the initial tables follow the (mutated) level when it is a valid one,
    // so that a rejection is never caused by a short table
    if (p.level_n != 5 && p.level_n <= 20 && p.d >= 1 && p.d <= CTM_MAXD && p.ic_terms == 1)
      fill(p, t, false);
    ctm_plan* plan = nullptr;
    const ctm_status st = ctm_plan_create(&p, &plan);
    CHECK(st == CTM_ERR_INVALID && plan == nullptr, "%s not rejected (status %d)", b.what, (int)st);
  }
  std::printf("ok   %zu invalid problems rejected\n", sizeof(bad) / sizeof(bad[0]));

  // enumeration, tables and shapes of every operator and size
  for (int d = 1; d <= 6; ++d) {
    ctm_problem p = base(d, d + 4, CTM_OP_HEAT);
    char what[64];
    std::snprintf(what, sizeof what, "heat d=%d n=%d", d, d + 4);
    create_cycle(p, what);
  }
  {
    ctm_problem p = base(6, 8, CTM_OP_VARCOEF);
    p.nsteps = 1024;
    p.mgrit_levels = 3;
    p.mgrit_cf = 8;
    p.prec = CTM_PREC_MIXED;
    create_cycle(p, "varcoef d=6 n=8, 3 levels, mixed");
  }
  {
    ctm_problem p = base(4, 8, CTM_OP_OU);
    p.nsteps = 512;
    p.mgrit_levels = 3;
    p.mgrit_cf = 4;
    create_cycle(p, "OU d=4 n=8");
  }
  {
    ctm_problem p = base(5, 6, CTM_OP_CME);
    p.nsteps = 256;
    create_cycle(p, "CME d=5 n=6 lattice");
  }
  {
    ctm_problem p = base(2, 14, CTM_OP_DRIFT);
    p.level_min = 6;
    p.nsteps = 256;
    create_cycle(p, "drift d=2 n=14 L0=6 (streaming grids)");
  }
  {
    ctm_problem p = base(3, 7, CTM_OP_HEAT);
    p.nrecomb = 4;
    create_cycle(p, "heat d=3 n=7, 4 recombination blocks");
  }
  {
    ctm_problem p = base(1, 6, CTM_OP_HEAT);
    p.mgrit_levels = 1;
    create_cycle(p, "heat d=1, time-sequential");
  }
  {
    ctm_problem p = base(2, 6, CTM_OP_HEAT);
    p.manufactured = CTM_MMS_HEAT;
    for (int i = 0; i < 2; ++i) {
      p.lo[i] = 0.0;
      p.hi[i] = 1.0;
    }
    create_cycle(p, "manufactured heat d=2");
  }
  for (int r = 0; r < 20; ++r) create_cycle(base(3, 6, CTM_OP_VARCOEF), "varcoef d=3 repeated");
  if (failures) {
    std::printf("%d failures\n", failures);
    return 1;
  }
  std::printf("all host checks passed\n");
  return 0;
}
