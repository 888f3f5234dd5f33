// Host side of the library: problem validation, enumeration of the
// combination index set, per-grid geometry and coefficient tables, the
// MGRIT driver and the C entry points declared in ctm.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "ctm_internal.h"

using namespace ctm;

namespace {

thread_local std::string g_last_error;

ctm_status fail(ctm_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

#define CTM_HIP(call)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return fail(CTM_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));            \
  } while (0)

struct GridHost {
  int lev[MAXD];
  int w;
  double coef;
  long long npts, off;
  double cost;
};

// All compositions of `total` into `parts` integers >= lmin, lexicographic.
void compositions(int total, int parts, int lmin, std::vector<int>& cur,
                  std::vector<std::vector<int>>& out) {
  if (parts == 1) {
    if (total >= lmin) {
      cur.push_back(total);
      out.push_back(cur);
      cur.pop_back();
    }
    return;
  }
  for (int first = lmin; first <= total - lmin * (parts - 1); ++first) {
    cur.push_back(first);
    compositions(total - first, parts - 1, lmin, cur, out);
    cur.pop_back();
  }
}

long long binom(int n, int k) {
  if (k < 0 || k > n) return 0;
  long long r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

}  // namespace

// Tasks (g, q) of one launch phase, grouped by the launch shape (size
// class) of their grid; inside a class, grids by decreasing cost.
struct TaskSet {
  int2* d = nullptr;
  long long total = 0;
  struct Range {
    int shape;
    long long offset, count;
    double points;  // unknowns summed over the range's tasks
  };
  std::vector<Range> ranges;
};

struct ctm_plan {
  ctm_problem prob;
  std::vector<double> icw, icf;
  int d = 0, n = 0, G = 0;
  long long slen = 0;
  int maxpts = 0;
  bool lattice = false;
  int opc = OPC_HEAT, solver = SOLV_CG;
  bool mixed = false;
  int shape = 0;
  int tabmax = 0;
  size_t smem_chain = 0;
  std::vector<GridHost> grids;
  std::vector<GridDev> hdev;
  std::vector<double> htab;
  std::vector<int> order;  // grid indices by decreasing estimated cost
  int device = 0;
  // device data owned by the plan
  GridDev* dgrids = nullptr;
  double* dtab = nullptr;
  long long* doffsets = nullptr;
  double* dicw = nullptr;
  double* dicf = nullptr;
  unsigned long long* dcounters = nullptr;
  double* dsync = nullptr;    // [0] residual max, [1] status word (int in low bytes)
  double* dnorm2 = nullptr;   // [G]
  double* hsync = nullptr;    // pinned mirror of dsync
  int2* didentity = nullptr;  // (g, 0) in canonical order
  int2* dgstage = nullptr;    // gather stages: runs of grids [x, y) of one LDS stage
  int ngstage = 0;
  std::vector<int> gshape;    // launch shape of each grid (size class)
  std::map<long long, TaskSet> tsets;  // M -> (g, q) tasks grouped by shape
  // side streams for concurrent size classes: with the caller's stream they
  // make four, the number of hardware queues HIP gives a process by default
  static constexpr int kSideStreams = 3;
  hipStream_t cstreams[kSideStreams] = {};
  // lane of each size class: 0 = the caller's stream, l > 0 = cstreams[l - 1].
  // Fixed per plan, so that consecutive phases of one class need no
  // cross-stream synchronisation.
  int lane_of[kNumShapes + 1] = {};
  // MGRIT phase schedule (ctm_plan_set_schedule): CTM_SCHED_AUTO, _JOINED
  // or _PER_CLASS
  int sched = CTM_SCHED_AUTO;
  // cyclic-reduction steps of the line preconditioner each size class's LDS
  // table must hold: the largest log2(lanes per line) over its grids
  int pcr_of[kNumShapes] = {};
  // coefficient-table doubles each size class's LDS must hold: the largest
  // table of its grids (the plan-wide largest would cost LDS, and with it
  // work-groups per CU, in classes whose grids have small tables)
  int tab_of[kNumShapes] = {};
  // hierarchical basis (built on first use): node id of every unknown; per
  // node, the unknowns of all grids that share its basis function
  double block_t0 = 0.0;     // start time of the recombination block being solved
  // streaming grids: scratch of kStreamVectors vectors of stream_ss doubles
  // for each of up to stream_tasks tasks
  long long stream_ss = 0, stream_tasks = 0;
  double* dstream = nullptr;
  // wide streaming solver: launch ranges of at most wide_max_tasks streaming
  // tasks spread every task over wide_pb (point-wise) / wide_lb (line)
  // work-groups; per-task state and partial sums for wide_cap tasks (every
  // streaming task of the plan); the poll's busy flags in mapped pinned memory
  // (default: every streaming launch; the one-work-group-per-task kernel
  // remains for comparison and for plans whose coefficient tables leave no
  // room for the line tiles in LDS)
  static constexpr int kWideMaxGridY = 65535;
  int wide_cap = 0;
  int wide_max_tasks = kWideMaxGridY;
  int wide_pb = 0, wide_lb = 0, wide_maxblk = 0;
  WideTask* dwide = nullptr;
  double* dwpart = nullptr;
  int* hwide = nullptr;      // [wide_cap] the poll's per-task busy flags
  int* hwide_dev = nullptr;
  int wide_est = 4;  // Krylov iterations launched per step before the first poll
  hipEvent_t wide_ev = nullptr;
  // MGRIT convergence on the device: dmg[0] = stopping iteration (0 while
  // running), dmg[2 it], dmg[2 it + 1] = residual and dmg[0] after iteration
  // it; hmg its pinned per-iteration mirror; skip = dmg while a block's
  // iterations are queued (launches past the stopping iteration do nothing)
  double* dmg = nullptr;
  double* hmg = nullptr;      // mapped pinned memory: written by the convergence kernel
  double* hmg_dev = nullptr;  // its device address
  const double* skip = nullptr;
  std::vector<hipEvent_t> it_events;
  int hnodes = 0;
  int* dhnode = nullptr;    // [slen]
  int* dhoff = nullptr;     // [hnodes + 1]
  int* dhidx = nullptr;     // [slen], grouped by node, canonical order inside a node
  double* dhcoef = nullptr; // [slen] combination coefficient of the entry's grid
  double* dhsg = nullptr;   // [hnodes] combined surpluses
  std::vector<hipEvent_t> sync_events;    // fork/join events
  // two-level Schwarz preconditioner (precond = CTM_PRECOND_SCHWARZ): grid
  // and subdomain records, index arrays, the owner grid of every subdomain,
  // and per MGRIT level the dense local and coarse inverses
  bool schwarz = false;
  SchwarzGrid* dsch_grid = nullptr;
  SchwarzSub* dsch_sub = nullptr;
  int* dsch_ints = nullptr;
  int* dsch_subgrid = nullptr;
  std::vector<double*> dsch_linv, dsch_cinv;
  long long sch_nsub = 0;
  int sch_nmax = 0, sch_nbmax = 0;
  ctm_stats stats;
  bool timing = false;
  std::vector<hipEvent_t> events;  // pairs (start, stop) per timed launch
  std::vector<int> event_shape;    // shape of each timed pair
  size_t events_used = 0;

  ~ctm_plan() {
    hipFree(dgrids);
    hipFree(dtab);
    hipFree(doffsets);
    hipFree(dicw);
    hipFree(dicf);
    hipFree(dcounters);
    hipFree(dsync);
    hipFree(dnorm2);
    hipFree(didentity);
    hipFree(dgstage);
    hipFree(dhnode);
    hipFree(dhoff);
    hipFree(dhidx);
    hipFree(dhcoef);
    hipFree(dhsg);
    hipFree(dstream);
    hipFree(dwide);
    hipFree(dwpart);
    if (hwide) hipHostFree(hwide);
    if (wide_ev) hipEventDestroy(wide_ev);
    hipFree(dmg);
    if (hmg) hipHostFree(hmg);
    for (auto e : it_events) hipEventDestroy(e);
    if (hsync) hipHostFree(hsync);
    for (auto& kv : tsets) hipFree(kv.second.d);
    for (auto e : events) hipEventDestroy(e);
    for (auto e : sync_events) hipEventDestroy(e);
    for (auto s : cstreams)
      if (s) hipStreamDestroy(s);
    hipFree(dsch_grid);
    hipFree(dsch_sub);
    hipFree(dsch_ints);
    hipFree(dsch_subgrid);
    for (auto p : dsch_linv) hipFree(p);
    for (auto p : dsch_cinv) hipFree(p);
  }
};

namespace {

double level_dt(const ctm_plan* P, int level) {
  double dt = (P->prob.t1 - P->prob.t0) / (double)P->prob.nsteps;
  for (int l = 0; l < level; ++l) dt *= P->prob.mgrit_cf;
  return dt;
}

// Coefficient tables of one grid. SEP (OU, CME): per axis the 1-D rows
// (Lo, D, Up) of L, unscaled; VAR: per axis the node sines sin(2 pi x_j)
// and the face sines sin(2 pi (x_j - h/2)), faces j = 0..n_i.
void build_tables(ctm_plan* P, const GridHost& gh, GridDev& gd) {
  const ctm_problem& p = P->prob;
  gd.tab0 = (long long)P->htab.size();
  int pos = 0;
  for (int i = 0; i < P->d; ++i) {
    const int ni = gd.n[i];
    const double h = gd.h[i];
    gd.tab[i] = pos;
    if (P->opc == OPC_SEP) {
      for (int part = 0; part < 3; ++part) {
        for (int j = 0; j < ni; ++j) {
          const double x = gd.lo[i] + (double)(j + gd.j0) * h;
          double lo = 0, dg = 0, up = 0;
          if (p.op == CTM_OP_OU) {
            // flux form with donor-cell drift, face velocity w = -theta x
            const double th = p.theta[i], D = 0.5 * p.sigma * p.sigma;
            const double wu = -th * (x + 0.5 * h), wd = -th * (x - 0.5 * h);
            dg = (std::max(wu, 0.0) - std::min(wd, 0.0)) / h + 2.0 * D / (h * h);
            up = std::min(wu, 0.0) / h - D / (h * h);
            lo = -std::max(wd, 0.0) / h - D / (h * h);
          } else {
            // immigration-death jump chain with spacing h; no births at the last state
            const double k = p.k[i], gm = p.gamma[i];
            const bool last = (j == ni - 1);
            dg = (last ? 0.0 : k / h) + gm * x / h;
            lo = -k / h;
            up = -gm * (x + h) / h;
          }
          P->htab.push_back(part == 0 ? lo : (part == 1 ? dg : up));
        }
      }
      pos += 3 * ni;
    } else if (P->opc == OPC_DRIFT) {
      // theta (row-major) and H once per grid, after the loop over axes
    } else if (P->opc == OPC_VAR) {
      for (int j = 0; j < ni; ++j) {
        const double x = gd.lo[i] + (double)(j + gd.j0) * h;
        P->htab.push_back(std::sin(2.0 * M_PI * x));
      }
      for (int j = 0; j <= ni; ++j) {
        const double x = gd.lo[i] + ((double)(j + gd.j0) - 0.5) * h;
        P->htab.push_back(std::sin(2.0 * M_PI * x));
      }
      pos += 2 * ni + 1;
    }
  }
  if (P->opc == OPC_DRIFT) {
    const int d = P->d;
    for (int i = 0; i < d * d; ++i) P->htab.push_back(p.drift[i]);
    for (int i = 0; i < d; ++i) P->htab.push_back(p.diffusion[i]);
    pos = d * d + d;
  }
  gd.tabsz = pos;
  (void)gh;
}

ctm_status validate(const ctm_problem* p) {
  if (!p) return fail(CTM_ERR_INVALID, "problem is NULL");
  if (p->d < 1 || p->d > CTM_MAXD) return fail(CTM_ERR_INVALID, "d must be in 1..8");
  if (p->level_min < 1) return fail(CTM_ERR_INVALID, "level_min must be >= 1");
  if (p->level_n < 1 || p->level_n + p->d - 1 > 30)
    return fail(CTM_ERR_INVALID, "level_n must satisfy 1 <= n and n + d - 1 <= 30");
  if (p->level_n + p->d - 1 < p->d * p->level_min)
    return fail(CTM_ERR_INVALID, "no component grid with l >= level_min");
  for (int i = 0; i < p->d; ++i)
    if (!(p->hi[i] > p->lo[i])) return fail(CTM_ERR_INVALID, "box must have hi > lo");
  // the enumerations arrive from C, where any int value can be stored: they
  // are read as ints (a C++ load of an out-of-range enumerator is undefined)
  auto as_int = [](const void* e) {
    int v;
    std::memcpy(&v, e, sizeof v);
    return v;
  };
  const int op = as_int(&p->op);
  if (op < CTM_OP_HEAT || op > CTM_OP_DRIFT) return fail(CTM_ERR_INVALID, "unknown operator");
  const int prec = as_int(&p->prec), kry = as_int(&p->krylov), relax = as_int(&p->relax),
            mms = as_int(&p->manufactured);
  if (prec != CTM_PREC_FP64 && prec != CTM_PREC_MIXED)
    return fail(CTM_ERR_INVALID, "unknown precision");
  if (kry < CTM_KRYLOV_AUTO || kry > CTM_KRYLOV_BICGSTAB)
    return fail(CTM_ERR_INVALID, "unknown Krylov method");
  if (relax != CTM_RELAX_F && relax != CTM_RELAX_FCF)
    return fail(CTM_ERR_INVALID, "unknown relaxation");
  if (mms != CTM_MMS_NONE && mms != CTM_MMS_HEAT)
    return fail(CTM_ERR_INVALID, "unknown manufactured problem");
  if (p->op == CTM_OP_CME)
    for (int i = 0; i < p->d; ++i) {
      const double span = p->hi[i] - p->lo[i];
      if (span != std::ldexp(1.0, p->level_n))
        return fail(CTM_ERR_INVALID, "lattice box needs hi - lo = 2^n");
      if (p->k[i] < 0 || p->gamma[i] < 0)
        return fail(CTM_ERR_INVALID, "rates must be nonnegative");
    }
  if (!(p->t1 > p->t0)) return fail(CTM_ERR_INVALID, "t1 must exceed t0");
  if (p->nsteps < 1) return fail(CTM_ERR_INVALID, "nsteps must be >= 1");
  if (p->nrecomb < 1 || p->nsteps % p->nrecomb)
    return fail(CTM_ERR_INVALID, "nrecomb must divide nsteps");
  if (p->mgrit_levels < 1 || p->mgrit_levels > 8)
    return fail(CTM_ERR_INVALID, "mgrit_levels must be in 1..8");
  if (p->mgrit_levels > 1) {
    if (p->mgrit_cf < 2) return fail(CTM_ERR_INVALID, "mgrit_cf must be >= 2");
    long long div = 1;
    for (int l = 1; l < p->mgrit_levels; ++l) div *= p->mgrit_cf;
    if ((p->nsteps / p->nrecomb) % div)
      return fail(CTM_ERR_INVALID, "steps per block must be divisible by cf^(levels-1)");
    if (!(p->mgrit_tol > 0) || p->mgrit_maxit < 1)
      return fail(CTM_ERR_INVALID, "mgrit_tol must be > 0 and mgrit_maxit >= 1");
  }
  if (!(p->krylov_tol > 0) || p->krylov_maxit < 1)
    return fail(CTM_ERR_INVALID, "krylov_tol must be > 0 and krylov_maxit >= 1");
  if (p->prec == CTM_PREC_MIXED &&
      (!(p->refine_tol > 0) || !(p->inner_tol > 0) || p->refine_maxit < 1))
    return fail(CTM_ERR_INVALID, "mixed precision needs refine_tol, inner_tol > 0, refine_maxit >= 1");
  if (!(p->coarse_tol >= 0) || !(p->coarse_tol < 1))
    return fail(CTM_ERR_INVALID, "coarse_tol must be in [0, 1)");
  if (p->residual_mode != 0 &&
      (p->residual_mode != 1 || p->mgrit_levels < 2 || !p->warm_start ||
       p->manufactured != CTM_MMS_NONE))
    return fail(CTM_ERR_INVALID,
                "residual_mode needs MGRIT (two or more levels), warm_start and no manufactured "
                "forcing");
  if (as_int(&p->precond) != CTM_PRECOND_LINE && as_int(&p->precond) != CTM_PRECOND_SCHWARZ)
    return fail(CTM_ERR_INVALID, "unknown preconditioner");
  if (p->precond == CTM_PRECOND_SCHWARZ) {
    if (p->schwarz_s < kSchwarzMinS || p->schwarz_s > kSchwarzMaxS)
      return fail(CTM_ERR_INVALID, "schwarz_s must be in 2..6");
    if (p->manufactured != CTM_MMS_NONE)
      return fail(CTM_ERR_INVALID, "the Schwarz preconditioner runs every grid on the streaming "
                                   "solver, which has no manufactured forcing");
  }
  if (p->op == CTM_OP_DRIFT) {
    for (int i = 0; i < p->d; ++i)
      if (!(p->diffusion[i] >= 0) || !std::isfinite(p->diffusion[i]))
        return fail(CTM_ERR_INVALID, "drift: diffusion must be finite and >= 0");
    for (int i = 0; i < p->d * p->d; ++i)
      if (!std::isfinite(p->drift[i])) return fail(CTM_ERR_INVALID, "drift: theta not finite");
  }
  if (p->manufactured != CTM_MMS_NONE) {
    if (p->manufactured != CTM_MMS_HEAT || p->op != CTM_OP_HEAT)
      return fail(CTM_ERR_INVALID, "manufactured: only the heat problem (op = heat)");
    for (int i = 0; i < p->d; ++i)
      if (p->lo[i] != 0.0 || p->hi[i] != 1.0)
        return fail(CTM_ERR_INVALID, "manufactured heat problem lives on [0,1]^d");
  }
  const bool sym = (p->op == CTM_OP_HEAT || p->op == CTM_OP_VARCOEF);
  if (p->krylov == CTM_KRYLOV_CG && !sym)
    return fail(CTM_ERR_INVALID, "CG needs a symmetric operator (heat or varcoef)");
  if (p->manufactured == CTM_MMS_NONE &&
      (p->ic_terms < 1 || p->ic_terms > CTM_MAX_IC_TERMS || !p->ic_weight || !p->ic_factor))
    return fail(CTM_ERR_INVALID, "initial value needs 1..16 terms with weight and factor arrays");
  if (p->manufactured != CTM_MMS_NONE &&
      (p->ic_terms < 0 || p->ic_terms > CTM_MAX_IC_TERMS ||
       (p->ic_terms > 0 && (!p->ic_weight || !p->ic_factor))))
    return fail(CTM_ERR_INVALID, "initial value arrays inconsistent with ic_terms");
  return CTM_OK;
}

// Lanes a grid needs in the line layout with K unknowns per lane.
int lanes_needed(const GridDev& gd, int K) {
  int lc = (gd.ns + K - 1) / K;
  int p = 1;
  while (p < lc) p <<= 1;
  return gd.nlines * p;
}

// Smallest K whose chunks keep every line of the grids inside one wave,
// then the smallest work-group that holds them all (or -1).
int pick_shape(const std::vector<GridDev>& gds) {
  int maxns = 0;
  for (auto& gd : gds) maxns = std::max(maxns, gd.ns);
  auto fits = [&](int s) {
    const int K = kShapes[s].K, W = kShapes[s].W;
    if (maxns > 64 * K) return false;
    for (auto& gd : gds)
      if (lanes_needed(gd, K) > 64 * W) return false;
    return true;
  };
  for (int K : {4, 8}) {
    if (maxns > 64 * K) continue;
    for (int s = 0; s < kNumShapes; ++s)
      if (kShapes[s].K == K && fits(s)) return s;
  }
  return -1;
}

// Shape with K unknowns per lane and the fewest waves that hold the lines
// of grid gd, or -1.
int min_waves_shape(const GridDev& gd, int K) {
  if (gd.ns > 64 * K) return -1;
  for (int s = 0; s < kNumShapes; ++s)
    if (kShapes[s].K == K && lanes_needed(gd, K) <= 64 * kShapes[s].W) return s;
  return -1;
}

// Default size class of one grid: K = 4 while its lines fit a wave (fewer
// registers, higher occupancy) and it needs at most 256 lanes (512 for the
// operators with per-line coefficients, whose K = 8 kernels need twice the
// registers of K = 4 and run one wave per SIMD), else 8; then the fewest
// waves that hold it. ctm_autotune revises it per anisotropy class.
int grid_shape(const GridDev& gd, bool heat) {
  const int s4 = min_waves_shape(gd, 4);
  if (s4 >= 0 && lanes_needed(gd, 4) > (heat ? 256 : 512)) {
    const int s8 = min_waves_shape(gd, 8);
    if (s8 >= 0) return s8;
  }
  return s4 >= 0 ? s4 : min_waves_shape(gd, 8);
}

// Cyclic-reduction steps of grid gd's lines with K unknowns per lane.
int pcr_steps(const GridDev& gd, int K) {
  int lc = 1, steps = 0;
  while (lc < (gd.ns + K - 1) / K) {
    lc <<= 1;
    ++steps;
  }
  return steps;
}

// LDS of one compute unit of gfx950: the most a work-group can allocate.
constexpr size_t kMaxLdsBytes = 160 * 1024;

// Whether grid gd's chain-kernel work-group fits the LDS in shape sh (its
// line preconditioner's table grows with log2 of the lanes per line).
// Whether a launch of shape sh keeps the FP64 line operator in LDS: the
// mixed K = 4 chains of the variable-coefficient operator (chain kernel).
bool parks_op(const ctm_plan* P, int sh, bool mixed) {
  return mixed && P->opc == OPC_VAR && sh < kNumShapes && kShapes[sh].K == 4;
}

// The chain kernel's static LDS (its copy of the grid descriptor) comes on
// top of the dynamic LDS. A mixed plan also launches its classes in FP64
// (the coarse MGRIT levels of coarse_in_fp64, the per-grid propagation),
// whose layout is larger (FP64 tables and cyclic-reduction rows): both must
// fit, or the FP64 launch is refused.
bool shape_fits(const ctm_plan* P, const GridDev& gd, int sh) {
  const int pcr = pcr_steps(gd, kShapes[sh].K);
  const bool heat = P->opc == OPC_HEAT;
  const size_t limit = kMaxLdsBytes - sizeof(GridDev);
  if (chain_smem_bytes(sh, P->tabmax, P->mixed, heat, pcr, parks_op(P, sh, P->mixed)) > limit)
    return false;
  return !P->mixed || chain_smem_bytes(sh, P->tabmax, false, heat, pcr, false) <= limit;
}

// The default shape of grid gd among those whose LDS fits, or -1 (streaming).
int grid_shape_fitting(const ctm_plan* P, const GridDev& gd) {
  const int sh = grid_shape(gd, P->opc == OPC_HEAT);
  if (sh < 0 || shape_fits(P, gd, sh)) return sh;
  const int alt = min_waves_shape(gd, kShapes[sh].K == 4 ? 8 : 4);
  return (alt >= 0 && shape_fits(P, gd, alt)) ? alt : -1;
}

ctm_status tasks_for(ctm_plan* P, long long M, TaskSet** out) {
  auto it = P->tsets.find(M);
  if (it != P->tsets.end()) {
    *out = &it->second;
    return CTM_OK;
  }
  TaskSet ts;
  std::vector<int2> t;
  t.reserve((size_t)P->G * M);
  for (int s = 0; s <= kStreamShape; ++s) {
    const long long start = (long long)t.size();
    double pts = 0.0;
    for (int g : P->order)
      if (P->gshape[g] == s) {
        for (long long q = 0; q < M; ++q) t.push_back(make_int2(g, (int)q));
        pts += (double)P->grids[g].npts * (double)M;
      }
    const long long cnt = (long long)t.size() - start;
    if (cnt) ts.ranges.push_back({s, start, cnt, pts});
  }
  ts.total = (long long)t.size();
  CTM_HIP(hipMalloc(&ts.d, t.size() * sizeof(int2)));
  CTM_HIP(hipMemcpy(ts.d, t.data(), t.size() * sizeof(int2), hipMemcpyHostToDevice));
  P->tsets[M] = ts;
  *out = &P->tsets[M];
  return CTM_OK;
}

// Lanes of the size classes: in decreasing order of unknowns, each class
// onto the lane (caller's stream or a side stream) with the fewest so far.
// Also refreshes the classes' cyclic-reduction table sizes.
void assign_lanes(ctm_plan* P) {
  for (int s = 0; s < kNumShapes; ++s) P->pcr_of[s] = P->tab_of[s] = 0;
  for (int g = 0; g < P->G; ++g) {
    const int s = P->gshape[g];
    if (s < kNumShapes) {
      P->pcr_of[s] = std::max(P->pcr_of[s], pcr_steps(P->hdev[g], kShapes[s].K));
      P->tab_of[s] = std::max(P->tab_of[s], P->hdev[g].tabsz);
    }
  }
  constexpr int nlanes = ctm_plan::kSideStreams + 1;
  double pts[kNumShapes + 1] = {};
  for (int g = 0; g < P->G; ++g) pts[P->gshape[g]] += (double)P->grids[g].npts;
  int order[kNumShapes + 1];
  for (int i = 0; i <= kNumShapes; ++i) order[i] = i;
  std::stable_sort(order, order + kNumShapes + 1, [&](int x, int y) { return pts[x] > pts[y]; });
  double load[nlanes] = {};
  for (int i : order) {
    int best = 0;
    for (int l = 1; l < nlanes; ++l)
      if (load[l] < load[best]) best = l;
    P->lane_of[i] = best;
    load[best] += pts[i];
  }
}

// Move grid g to size class sh; the cached task lists are rebuilt on next use.
void set_shape(ctm_plan* P, int g, int sh) {
  if (P->gshape[g] == sh) return;
  P->gshape[g] = sh;
  for (auto& kv : P->tsets) hipFree(kv.second.d);
  P->tsets.clear();
  assign_lanes(P);
}

// The Schwarz preconditioner of MGRIT level `level` (empty without it).
SchwarzView schwarz_view(const ctm_plan* P, int level) {
  SchwarzView v;
  std::memset(&v, 0, sizeof(v));
  if (!P->schwarz || level < 0 || level >= (int)P->dsch_linv.size()) return v;
  v.grid = P->dsch_grid;
  v.sub = P->dsch_sub;
  v.ints = P->dsch_ints;
  v.linv = P->dsch_linv[level];
  v.cinv = P->dsch_cinv[level];
  v.balanced = (P->solver == SOLV_CG) ? 1 : 0;
  v.nbmax = P->sch_nbmax;
  return v;
}

// mgrit: arguments of an MGRIT relaxation or coarse chain (residual mode
// applies there only; plain time stepping always solves to tolerance).
ChainArgs base_args(ctm_plan* P, int level, int nsteps, bool fp64_only = false,
                    bool mgrit = false) {
  ChainArgs a;
  std::memset(&a, 0, sizeof(a));
  a.grids = P->dgrids;
  a.tab64 = P->dtab;
  a.amp = P->prob.amp;
  a.dt = level_dt(P, level);
  a.slen = P->slen;
  a.nsteps = nsteps;
  a.maxit = P->prob.krylov_maxit;
  a.refine_maxit = P->prob.refine_maxit;
  const bool mixed = P->mixed && !fp64_only;
  a.tol = mixed ? P->prob.refine_tol : P->prob.krylov_tol;
  a.inner_tol = P->prob.inner_tol;
  a.status = reinterpret_cast<int*>(P->dsync + 1);
  a.skip = P->skip;
  a.sch = schwarz_view(P, level);
  if (mgrit && P->prob.residual_mode) {  // fixed-count steps on every level
    a.resmode = 1;
    a.tol = 0.0;
  }
  // the forcing enters the level-0 steps only (coarse levels solve for
  // corrections, whose right-hand sides are residuals)
  if (level == 0 && P->prob.manufactured == CTM_MMS_HEAT) {
    a.fkind = 1;
    a.ft0 = P->block_t0;
    a.ftq = 0.0;
  }
  return a;
}

// Whether the coarse MGRIT levels of a mixed plan run the FP64 kernels: for
// the operators with per-line coefficients, whose mixed kernels hold both
// precisions' coefficients and run one wave per SIMD against two for FP64,
// when the coarse tolerance is loose (the coarse steps only steer the
// correction; warm-started FP64 steps meet 1e-3 in about one iteration).
// Measured on the 6-D workload: 1.46 -> 1.23 s per mixed solve, with 10
// MGRIT iterations instead of 11; on the 3-D heat workload (low-register
// kernels) the single FP32 coarse solves stay faster.
bool coarse_in_fp64(const ctm_plan* P) {
  return P->mixed && P->opc != OPC_HEAT && P->prob.coarse_tol >= 1e-5 && !P->prob.residual_mode;
}

// Arguments of a chain on MGRIT level l >= 1: the coarse tolerance, when set,
// replaces the level-0 one. In the mixed path a tolerance that FP32 reaches
// by itself (>= 1e-5) makes each coarse step a single FP32 solve (heat) or an
// FP64 solve (coarse_in_fp64); otherwise the inner FP32 target follows it.
ChainArgs coarse_args(ctm_plan* P, int level, int nsteps) {
  const bool c64 = coarse_in_fp64(P);
  ChainArgs a = base_args(P, level, nsteps, c64, true);
  const double ct = P->prob.coarse_tol;
  if (ct > 0 && !a.resmode) {
    a.tol = ct;
    a.inner_tol = std::max(P->prob.inner_tol, 0.25 * ct);
    if (P->mixed && ct >= 1e-5 && !c64) {
      a.single32 = 1;
      a.inner_tol = ct;
    }
  }
  return a;
}

VecRef vref(double* base, long long a, long long b) { return VecRef{base, a, b}; }

// Vectors one task must read or write once: start, optional write-back,
// per-step forcing, initial guesses and intermediate stores, final store and
// residual target.
double chain_vectors_per_task(const ChainArgs& a) {
  double v = 0;
  if (a.start.base) v += 1;
  if (a.start_wb.base) v += 1;
  if (a.forcing.base) v += a.nsteps;
  if (a.inter.base) v += a.nsteps - 1;
  if (a.fin.base) v += 1;
  if (a.target.base) v += 1;
  if (a.guess.base) v += a.nsteps - 1;
  if (a.guess_fin.base) v += 1;
  return v;
}

hipEvent_t take_event(ctm_plan* P, size_t& used, std::vector<hipEvent_t>& pool, bool timed) {
  while (pool.size() <= used) {
    hipEvent_t ev = nullptr;
    if (hipEventCreateWithFlags(&ev, timed ? hipEventDefault : hipEventDisableTiming) !=
        hipSuccess)
      return nullptr;
    pool.push_back(ev);
  }
  return pool[used++];
}

// Whether a launch range runs on the wide streaming solver.
bool use_wide(const ctm_plan* P, int shape, long long count) {
  return shape == kStreamShape && !P->schwarz && count > 0 && count <= P->wide_max_tasks &&
         count <= P->wide_cap &&
         (size_t)P->tabmax * sizeof(double) + kWideStaticLds <= 65536;
}

// The chain of a launch range on the wide solver: per step, the step
// transition, the initial residual and Krylov iterations in batches; after a
// batch, a poll kernel applies the next stopping test and the host waits for
// its per-task busy flags (the only host synchronisation), then launches
// more iterations or the next step. The first batch of a step has as many
// iterations as the previous step needed. Residual mode iterates a fixed
// count and never waits.
ctm_status run_wide(ctm_plan* P, const ChainArgs& c, int count, hipStream_t s) {
  WideArgs w{};
  w.a = c;
  w.scratch = P->dstream;
  w.ss = P->stream_ss;
  w.st = P->dwide;
  w.part = P->dwpart;
  w.maxblk = P->wide_maxblk;
  w.host_out = P->hwide_dev;
  w.stage = count > 64;  // (LDS-staged line sweeps on launches of many tasks)
  const dim3 gp(P->wide_pb, count), gl(P->wide_lb, count);
  const bool bicg = (P->solver == SOLV_BICG);
  const bool res = c.resmode != 0;
  auto go = [&](int kind, dim3 grid) -> ctm_status {
    const hipError_t e = launch_wide(P->opc, P->solver, P->d, kind, w, grid, P->tabmax, s);
    if (e != hipSuccess) return fail(CTM_ERR_HIP, std::string("wide launch: ") + hipGetErrorString(e));
    return CTM_OK;
  };
  ctm_status st;
  if ((st = go(WK_SETUP, gl)) != CTM_OK) return st;
  int prev = 0;
  for (int j = 1; j <= c.nsteps; ++j) {
    w.j = j;
    w.prev_its = prev;
    if ((st = go(WK_STEP, gp)) != CTM_OK) return st;
    if (res && j == c.nsteps && c.target.base) break;  // the step kernel formed the residual
    if ((st = go(WK_INIT, gp)) != CTM_OK) return st;
    int i = 1;  // next iteration
    if (bicg) {
      w.i = 1;
      if ((st = go(WK_BA, gl)) != CTM_OK) return st;
    }
    int budget = res ? c.maxit : std::max(1, std::min(c.maxit, P->wide_est));
    for (;;) {
      for (int n = 0; n < budget && i <= c.maxit; ++n, ++i) {
        w.i = i;
        if (bicg) {
          if ((st = go(WK_BB, gp)) != CTM_OK) return st;
          if ((st = go(WK_BC, gl)) != CTM_OK) return st;
          if ((st = go(WK_BD, gp)) != CTM_OK) return st;
          w.i = i + 1;
          if ((st = go(WK_BA, gl)) != CTM_OK) return st;
        } else {
          if ((st = go(WK_CA, gl)) != CTM_OK) return st;
          if ((st = go(WK_CB, gp)) != CTM_OK) return st;
          if ((st = go(WK_CC, gp)) != CTM_OK) return st;
        }
      }
      w.i = i;
      if ((st = go(WK_POLL, dim3(1, count))) != CTM_OK) return st;
      if (res || i > c.maxit) break;
      CTM_HIP(hipEventRecord(P->wide_ev, s));
      CTM_HIP(hipEventSynchronize(P->wide_ev));
      int busy = 0;
      for (int t = 0; t < count; ++t) busy += __atomic_load_n(P->hwide + t, __ATOMIC_ACQUIRE);
      if (busy == 0) break;
      budget = std::max(1, (i - 1) / 4);
    }
    prev = i - 1;
    if (!res) P->wide_est = std::max(1, prev);
  }
  w.j = c.nsteps;
  w.prev_its = prev;
  if ((st = go(WK_FIN, gp)) != CTM_OK) return st;
  return go(WK_FINISH, dim3(1, count));
}

// One launch of the chain kernel for the tasks [offset, offset + count) of a
// task array, all of one shape, on stream s.
ctm_status launch_range(ctm_plan* P, const ChainArgs& a, const int2* tasks, int shape,
                        long long offset, long long count, double points, hipStream_t s,
                        bool mixed) {
  ChainArgs c = a;
  c.tasks = tasks + offset;
  if (a.res2) c.res2 = a.res2 + offset;
  const bool wide = use_wide(P, shape, count);
  // statistics slot: the size class, the wide solver, or the FP64 launches
  // of a mixed plan
  const int slot = wide ? kWideSlot
                        : (P->mixed && !mixed && shape != kStreamShape) ? kCoarse64Slot : shape;
  c.counters = P->dcounters + (size_t)slot * CNT_N;
  c.pcrmax = (shape == kStreamShape) ? 0 : P->pcr_of[shape];
  const size_t smem = (shape == kStreamShape)
                          ? 0
                          : chain_smem_bytes(shape, P->tab_of[shape], mixed, P->opc == OPC_HEAT,
                                             c.pcrmax, parks_op(P, shape, mixed));
  // algorithmic bytes: every vector role of every task once
  P->stats.shape_bytes[slot] += 8.0 * points * chain_vectors_per_task(a);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (P->timing) {
    e0 = take_event(P, P->events_used, P->events, true);
    e1 = take_event(P, P->events_used, P->events, true);
    if (!e0 || !e1) return fail(CTM_ERR_HIP, "event creation failed");
    P->event_shape.resize(P->events.size());
    P->event_shape[P->events_used - 2] = slot;
    CTM_HIP(hipEventRecord(e0, s));
  }
  hipError_t e;
  if (shape == kStreamShape) {
    if (count > P->stream_tasks) return fail(CTM_ERR_INVALID, "streaming launch exceeds its scratch");
    if (wide) {
      ctm_status st = run_wide(P, c, (int)count, s);
      if (st != CTM_OK) return st;
      e = hipSuccess;
    } else {
      e = launch_stream(P->opc, P->solver, P->d, c, (int)count, P->tabmax, P->dstream,
                        P->stream_ss, s);
    }
  } else {
    e = launch_chain(P->opc, P->solver, mixed, shape, c, (int)count, smem, P->tab_of[shape], s);
  }
  if (e != hipSuccess) {
    char what[160];
    if (shape == kStreamShape)
      std::snprintf(what, sizeof what, "streaming, %lld tasks", count);
    else
      std::snprintf(what, sizeof what, "shape W%dK%d, %s, %zu B of LDS, %lld tasks",
                    kShapes[shape].W, kShapes[shape].K, mixed ? "mixed" : "FP64", smem, count);
    return fail(CTM_ERR_HIP, std::string("chain launch (") + what + "): " + hipGetErrorString(e));
  }
  if (P->timing) CTM_HIP(hipEventRecord(e1, s));
  P->stats.chain_launches += 1;
  return CTM_OK;
}

// Stream of lane l: the caller's stream s for l = 0 (may be the null
// stream), else side stream l - 1, created on first use.
ctm_status lane_stream(ctm_plan* P, int l, hipStream_t s, hipStream_t* out) {
  if (l > 0 && !P->cstreams[l - 1])
    CTM_HIP(hipStreamCreateWithFlags(&P->cstreams[l - 1], hipStreamNonBlocking));
  *out = (l == 0) ? s : P->cstreams[l - 1];
  return CTM_OK;
}

// Make stream s wait for all work queued on the side streams.
ctm_status join_lanes(ctm_plan* P, hipStream_t s) {
  size_t used = 0;
  for (int l = 1; l <= ctm_plan::kSideStreams; ++l) {
    if (!P->cstreams[l - 1]) continue;
    hipEvent_t j = take_event(P, used, P->sync_events, false);
    if (!j) return fail(CTM_ERR_HIP, "event creation failed");
    CTM_HIP(hipEventRecord(j, P->cstreams[l - 1]));
    CTM_HIP(hipStreamWaitEvent(s, j, 0));
  }
  return CTM_OK;
}

// Launch a phase: one kernel per size class, each on its class's lane (the
// caller's stream or a side stream), so that the classes run concurrently.
// fork: the side streams first wait for the work queued on s; without it
// they continue from their own previous phase (valid when every task of the
// phase reads only what its own class wrote before, or what was joined and
// forked earlier). join: s then waits for the side streams.
ctm_status run_chain(ctm_plan* P, const ChainArgs& a, const TaskSet& ts, hipStream_t s,
                     bool fp64_only = false, bool fork = true, bool join = true) {
  const bool mixed = P->mixed && !fp64_only;
  // algorithmic bytes: every vector of every task once
  const double per_grid_sets = (double)ts.total / (double)P->G;
  P->stats.chain_bytes += 8.0 * (double)P->slen * per_grid_sets * chain_vectors_per_task(a);
  constexpr int nlanes = ctm_plan::kSideStreams + 1;
  // launch order: decreasing work (unknowns x tasks)
  std::vector<int> order(ts.ranges.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  // (ranges on the wide solver wait for their poll on the host: they go last,
  // once everything else of the phase is queued)
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    const bool wx = use_wide(P, ts.ranges[x].shape, ts.ranges[x].count);
    const bool wy = use_wide(P, ts.ranges[y].shape, ts.ranges[y].count);
    if (wx != wy) return wy;
    return ts.ranges[x].points > ts.ranges[y].points;
  });
  size_t used = 0;
  // the fork point is recorded before anything of this phase is queued on s
  hipEvent_t fork_ev = nullptr;
  bool side = false;
  for (const auto& r : ts.ranges) side |= (P->lane_of[r.shape] > 0);
  if (fork && side) {
    fork_ev = take_event(P, used, P->sync_events, false);
    if (!fork_ev) return fail(CTM_ERR_HIP, "event creation failed");
    CTM_HIP(hipEventRecord(fork_ev, s));
  }
  bool used_lane[nlanes] = {};
  for (int i : order) {
    const auto& r = ts.ranges[i];
    const int l = P->lane_of[r.shape];
    hipStream_t cs = nullptr;
    ctm_status st = lane_stream(P, l, s, &cs);
    if (st != CTM_OK) return st;
    if (l > 0 && fork && !used_lane[l]) CTM_HIP(hipStreamWaitEvent(cs, fork_ev, 0));
    used_lane[l] = true;
    st = launch_range(P, a, ts.d, r.shape, r.offset, r.count, r.points, cs, mixed);
    if (st != CTM_OK) return st;
  }
  if (!join) return CTM_OK;
  for (int l = 1; l < nlanes; ++l) {
    if (!used_lane[l]) continue;
    hipEvent_t j = take_event(P, used, P->sync_events, false);
    if (!j) return fail(CTM_ERR_HIP, "event creation failed");
    CTM_HIP(hipEventRecord(j, P->cstreams[l - 1]));
    CTM_HIP(hipStreamWaitEvent(s, j, 0));
  }
  return CTM_OK;
}

// The plain reference schedule: one grid, one launch.
ctm_status run_chain_grid(ctm_plan* P, const ChainArgs& a, int g, hipStream_t s) {
  P->stats.chain_bytes += 8.0 * (double)P->grids[g].npts * chain_vectors_per_task(a);
  return launch_range(P, a, P->didentity, P->gshape[g], g, 1, (double)P->grids[g].npts, s,
                      false);
}

// Sum of the timed launch durations (after the stream has been synchronised).
ctm_status accumulate_timing(ctm_plan* P) {
  double ms = 0.0;
  for (size_t i = 0; i + 1 < P->events_used; i += 2) {
    float t = 0.0f;
    CTM_HIP(hipEventElapsedTime(&t, P->events[i], P->events[i + 1]));
    ms += t;
    const int sh = P->event_shape[i];
    P->stats.shape_ms[sh] += t;
    P->stats.shape_launches[sh] += 1;
  }
  P->stats.chain_ms += ms;
  P->events_used = 0;
  return CTM_OK;
}

void reset_stats(ctm_plan* P) {
  std::memset(&P->stats, 0, sizeof(P->stats));
  P->events_used = 0;
}

// (a fill kernel rather than hipMemsetAsync: the counters are 8-byte words,
// and all-zero bits are a zero of either type)
ctm_status reset_device_stats(ctm_plan* P, hipStream_t s) {
  CTM_HIP(launch_fill_zero(reinterpret_cast<double*>(P->dcounters), (long long)kStatSlots * CNT_N, s));
  CTM_HIP(launch_fill_zero(P->dsync, 2, s));
  return CTM_OK;
}

// Fold the per-class device counters into the statistics.
void fold_counters(const ctm_plan* P, const unsigned long long* c, ctm_stats* st) {
  st->krylov_iterations = st->krylov_max = st->refine_sweeps = st->refine_max = 0;
  st->phi_solves = st->krylov_work = 0;
  for (int s = 0; s < kStatSlots; ++s) {
    const unsigned long long* k = c + (size_t)s * CNT_N;
    st->krylov_iterations += (long long)k[CNT_KRYLOV];
    st->krylov_max = std::max(st->krylov_max, (long long)k[CNT_KRYLOV_MAX]);
    st->refine_sweeps += (long long)k[CNT_REFINE];
    st->refine_max = std::max(st->refine_max, (long long)k[CNT_REFINE_MAX]);
    st->phi_solves += (long long)k[CNT_SOLVES];
    st->krylov_work += (long long)k[CNT_WORK];
    st->shape_work[s] = (long long)k[CNT_WORK];
    st->shape_dofsteps[s] = (long long)k[CNT_DOFSTEPS];
    // streaming: K = 0, and W = 16 (1,024 threads per task) or the wide
    // solver's kWW waves per work-group
    st->shape_w[s] = (s == kStreamShape)   ? 16
                     : (s == kWideSlot)    ? kWW
                     : (s == kCoarse64Slot) ? 0
                                            : kShapes[s].W;
    st->shape_k[s] = (s >= kStreamShape) ? 0 : kShapes[s].K;
  }
  (void)P;
}

ctm_status collect_device_stats(ctm_plan* P, hipStream_t s) {
  unsigned long long c[kStatSlots * CNT_N];
  CTM_HIP(hipMemcpyAsync(c, P->dcounters, sizeof(c), hipMemcpyDeviceToHost, s));
  CTM_HIP(hipMemcpyAsync(P->hsync, P->dsync, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  CTM_HIP(hipStreamSynchronize(s));
  fold_counters(P, c, &P->stats);
  P->stats.status_flags = *reinterpret_cast<int*>(P->hsync + 1);
  return accumulate_timing(P);
}

ctm_status status_from_flags(int flags) {
  if (flags & (1 << CTM_ERR_INVALID))
    return fail(CTM_ERR_INVALID, "a launch's cyclic-reduction table was too small for a grid");
  if (flags & (1 << CTM_ERR_NONFINITE)) return fail(CTM_ERR_NONFINITE, "non-finite value in a solve");
  if (flags & (1 << CTM_ERR_BREAKDOWN)) return fail(CTM_ERR_BREAKDOWN, "BiCGStab breakdown");
  if (flags & (1 << CTM_ERR_NOCONV)) return fail(CTM_ERR_NOCONV, "an implicit solve did not converge");
  return CTM_OK;
}

// ------------------------------------------------------------- MGRIT
// Workspace layout for one block (all vectors packed, float64):
//   U, Un     level-0 C-points, (M0 + 1) vectors each (Un only with FCF)
//   R[l]      residual on level l-1's C-points = right-hand side of level l, l >= 1
//   E[l]      all points of level l >= 1 (N_l + 1 vectors)
//   Cn[l]     C-relaxed C-points of level l (1 <= l < L-1, FCF)
//   X, Y      block start / end states; res2 per task; scalars
struct Layout {
  int L;
  long long c;
  std::vector<long long> N;  // N[l], steps on level l
  double* U = nullptr;
  double* Un = nullptr;
  double* Tr = nullptr;  // level-0 trajectory (warm starts), index c * q + j
  std::vector<double*> R, E, Cn;
  double* X = nullptr;
  double* Y = nullptr;
  double* res2 = nullptr;
  double* rpart = nullptr;  // partial maxima of the residual test
  size_t bytes = 0;
};

Layout make_layout(const ctm_plan* P, char* base) {
  Layout lay;
  const ctm_problem& p = P->prob;
  lay.L = p.mgrit_levels;
  lay.c = p.mgrit_cf;
  const long long Nb = p.nsteps / p.nrecomb;
  lay.N.resize(lay.L);
  lay.N[0] = Nb;
  for (int l = 1; l < lay.L; ++l) lay.N[l] = lay.N[l - 1] / lay.c;
  lay.R.assign(lay.L + 1, nullptr);
  lay.E.assign(lay.L + 1, nullptr);
  lay.Cn.assign(lay.L + 1, nullptr);
  size_t off = 0;
  const size_t vb = (size_t)P->slen * sizeof(double);
  auto take = [&](long long nvec) {
    double* ptr = base ? reinterpret_cast<double*>(base + off) : nullptr;
    off += (size_t)nvec * vb;
    off = (off + 255) & ~size_t(255);
    return ptr;
  };
  const bool fcf = (p.relax == CTM_RELAX_FCF);
  if (lay.L > 1) {
    const long long M0 = lay.N[0] / lay.c;
    lay.U = take(M0 + 1);
    if (fcf) lay.Un = take(M0 + 1);
    if (p.warm_start) lay.Tr = take(lay.N[0]);
    for (int l = 1; l < lay.L; ++l) {
      lay.R[l] = take(lay.N[l] + 1);
      lay.E[l] = take(lay.N[l] + 1);
      if (l < lay.L - 1 && fcf) lay.Cn[l] = take(lay.N[l] / lay.c + 1);
    }
  }
  lay.X = take(1);
  lay.Y = take(1);
  const long long maxtasks = (long long)P->G * std::max<long long>(1, lay.N[0] / std::max<long long>(1, lay.c));
  double* r2 = base ? reinterpret_cast<double*>(base + off) : nullptr;
  off += (size_t)maxtasks * sizeof(double);
  off = (off + 255) & ~size_t(255);
  lay.res2 = r2;
  lay.rpart = base ? reinterpret_cast<double*>(base + off) : nullptr;
  off += (size_t)kResBlocks * sizeof(double);
  off = (off + 255) & ~size_t(255);
  lay.bytes = off;
  return lay;
}

// One cycle on level l >= 1 for e_0 = g_0, e_n = Phi_l e_{n-1} + g_n from a
// zero initial guess; writes all points of E[l].
// dst = x + y (either may be null) on vectors q = 0..nvec-1, per size class
// on the class's lane, restricted to the class's grids.
ctm_status class_vec_add(ctm_plan* P, VecRef dst, VecRef x, VecRef y, long long nvec,
                         hipStream_t s) {
  TaskSet* single = nullptr;
  ctm_status st = tasks_for(P, 1, &single);
  if (st != CTM_OK) return st;
  for (const auto& r : single->ranges) {
    hipStream_t cs = nullptr;
    if ((st = lane_stream(P, P->lane_of[r.shape], s, &cs)) != CTM_OK) return st;
    CTM_HIP(launch_class_vec_add(single->d + r.offset, (int)r.count, P->dgrids, dst, x, y,
                                 (int)nvec, P->slen, cs, P->skip));
  }
  return CTM_OK;
}

// Every side lane waits for the work queued on s so far.
ctm_status fork_lanes(ctm_plan* P, hipStream_t s) {
  size_t used = 0;
  hipEvent_t ev = take_event(P, used, P->sync_events, false);
  if (!ev) return fail(CTM_ERR_HIP, "event creation failed");
  CTM_HIP(hipEventRecord(ev, s));
  for (int l = 1; l <= ctm_plan::kSideStreams; ++l) {
    hipStream_t cs = nullptr;
    ctm_status st = lane_stream(P, l, s, &cs);
    if (st != CTM_OK) return st;
    CTM_HIP(hipStreamWaitEvent(cs, ev, 0));
  }
  return CTM_OK;
}

// One MGRIT cycle on level l >= 1 for the residual equation. On the last
// level, e_m for m >= 1 is written and e_0 (= 0, cleared once per block) is
// left alone. per_class: every phase, fill and correction runs per size
// class on the lanes forked before, without a join (each reads only what its
// own class wrote); otherwise every phase is forked from and joined back
// into s. The first residual vector r_0 of every level is cleared once per
// block.
ctm_status cycle(ctm_plan* P, Layout& lay, int l, hipStream_t s, bool per_class) {
  const long long c = lay.c;
  double* G = lay.R[l];
  double* E = lay.E[l];
  const bool c64 = coarse_in_fp64(P);
  const bool fj = !per_class;  // fork and join around each phase
  ctm_status st;
  if (l == lay.L - 1) {
    ChainArgs a = coarse_args(P, l, (int)lay.N[l]);
    a.start = vref(nullptr, 0, 0);
    a.forcing = vref(G, 0, 0);
    a.inter = vref(E, 0, 0);
    a.fin = vref(E, 0, lay.N[l]);
    TaskSet* single = nullptr;
    if ((st = tasks_for(P, 1, &single)) != CTM_OK) return st;
    return run_chain(P, a, *single, s, c64, fj, fj);
  }
  const long long M = lay.N[l] / c;
  TaskSet* tasks = nullptr;
  if ((st = tasks_for(P, M, &tasks)) != CTM_OK) return st;
  // dst = x + y over nvec vectors: whole vectors on s, or per class
  auto add = [&](VecRef dst, VecRef x, VecRef y, long long nvec) -> ctm_status {
    if (per_class) return class_vec_add(P, dst, x, y, nvec, s);
    if (!x.base && !y.base) {
      CTM_HIP(launch_fill_zero(dst.base + dst.b * P->slen, nvec * P->slen, s, P->skip));
    } else {
      CTM_HIP(launch_vec_add(dst, x, y, (int)nvec, P->slen, s, P->skip));
    }
    return CTM_OK;
  };
  const VecRef none = vref(nullptr, 0, 0);
  if ((st = add(vref(E, 1, 0), none, none, lay.N[l] + 1)) != CTM_OK) return st;
  double* csrc;
  long long ca;
  if (P->prob.relax == CTM_RELAX_FCF) {
    double* Cn = lay.Cn[l];
    if ((st = add(vref(Cn, 1, 0), none, none, 1)) != CTM_OK) return st;
    ChainArgs fc = coarse_args(P, l, (int)c);
    fc.start = vref(E, c, 0);
    fc.forcing = vref(G, c, 0);
    fc.inter = vref(E, c, 0);
    fc.fin = vref(Cn, 1, 1);
    if ((st = run_chain(P, fc, *tasks, s, c64, fj, fj)) != CTM_OK) return st;
    ChainArgs fr = coarse_args(P, l, (int)c);
    fr.start = vref(Cn, 1, 0);
    fr.start_wb = vref(E, c, 0);
    fr.forcing = vref(G, c, 0);
    fr.inter = vref(E, c, 0);
    fr.fin = vref(lay.R[l + 1], 1, 1);
    fr.target = vref(Cn, 1, 1);
    if ((st = run_chain(P, fr, *tasks, s, c64, fj, fj)) != CTM_OK) return st;
    csrc = Cn;
    ca = 1;
  } else {
    ChainArgs fr = coarse_args(P, l, (int)c);
    fr.start = vref(E, c, 0);
    fr.forcing = vref(G, c, 0);
    fr.inter = vref(E, c, 0);
    fr.fin = vref(lay.R[l + 1], 1, 1);
    fr.target = vref(E, c, c);
    if ((st = run_chain(P, fr, *tasks, s, c64, fj, fj)) != CTM_OK) return st;
    csrc = E;
    ca = c;
  }
  if ((st = cycle(P, lay, l + 1, s, per_class)) != CTM_OK) return st;
  // correction at the C-points, then F-relaxation (ideal interpolation)
  if ((st = add(vref(E, c, 0), vref(csrc, ca, 0), vref(lay.E[l + 1], 1, 0), M + 1)) != CTM_OK)
    return st;
  ChainArgs fi = coarse_args(P, l, (int)(c - 1));
  fi.start = vref(E, c, 0);
  fi.forcing = vref(G, c, 0);
  fi.inter = vref(E, c, 0);
  fi.fin = vref(E, c, c - 1);
  return run_chain(P, fi, *tasks, s, c64, fj, fj);
}

// Node map of the hierarchical basis: every unknown named by its node on
// the finest grid (per axis J * 2^(n - l_i)); unknowns of different grids at
// the same node share one hierarchical basis function (Section 2.2.2).
ctm_status ensure_hier(ctm_plan* P) {
  if (P->dhnode) return CTM_OK;
  const long long N = P->slen;
  if (N >= (1LL << 31)) return fail(CTM_ERR_INVALID, "state too long for the node map");
  const int d = P->d;
  std::vector<uint32_t> J((size_t)N * d);
  std::vector<double> cof((size_t)N);
  for (const auto& g : P->hdev) {
    for (int p = 0; p < g.npts; ++p) {
      int rem = p;
      for (int i = d - 1; i >= 0; --i) {
        const int j = rem % g.n[i];
        rem /= g.n[i];
        J[(size_t)(g.off + p) * d + i] = (uint32_t)(j + g.j0) << (P->n - g.lev[i]);
      }
      cof[(size_t)(g.off + p)] = g.coef;
    }
  }
  std::vector<int> ord((size_t)N);
  for (long long p = 0; p < N; ++p) ord[(size_t)p] = (int)p;
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
    const uint32_t* x = &J[(size_t)a * d];
    const uint32_t* y = &J[(size_t)b * d];
    for (int i = 0; i < d; ++i)
      if (x[i] != y[i]) return x[i] < y[i];
    return false;
  });
  std::vector<int> node((size_t)N), off;
  std::vector<double> coef((size_t)N);
  for (size_t e = 0; e < ord.size(); ++e) {
    const bool fresh = (e == 0) || std::memcmp(&J[(size_t)ord[e] * d], &J[(size_t)ord[e - 1] * d],
                                               d * sizeof(uint32_t)) != 0;
    if (fresh) off.push_back((int)e);
    node[(size_t)ord[e]] = (int)off.size() - 1;
    coef[e] = cof[(size_t)ord[e]];
  }
  off.push_back((int)N);
  const int nodes = (int)off.size() - 1;
  // every table is allocated into a local first and handed to the plan only
  // once all of them exist (dhnode, the "built" marker, last), so that a
  // failed allocation leaves nothing behind and a later call starts over
  void* bufs[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  const size_t bytes[5] = {off.size() * sizeof(int), ord.size() * sizeof(int),
                           coef.size() * sizeof(double), (size_t)nodes * sizeof(double),
                           node.size() * sizeof(int)};
  const void* src[5] = {off.data(), ord.data(), coef.data(), nullptr, node.data()};
  for (int i = 0; i < 5; ++i) {
    ctm_status st = CTM_OK;
    if (hipMalloc(&bufs[i], bytes[i]) != hipSuccess) {
      bufs[i] = nullptr;
      st = fail(CTM_ERR_NOMEM, "device allocation failed");
    } else if (src[i] && hipMemcpy(bufs[i], src[i], bytes[i], hipMemcpyHostToDevice) != hipSuccess) {
      st = fail(CTM_ERR_HIP, "hipMemcpy failed");
    }
    if (st != CTM_OK) {
      for (int k = 0; k <= i; ++k) hipFree(bufs[k]);
      return st;
    }
  }
  P->dhoff = static_cast<int*>(bufs[0]);
  P->dhidx = static_cast<int*>(bufs[1]);
  P->dhcoef = static_cast<double*>(bufs[2]);
  P->dhsg = static_cast<double*>(bufs[3]);
  P->dhnode = static_cast<int*>(bufs[4]);
  P->hnodes = nodes;
  return CTM_OK;
}

// Combine-then-project through the hierarchical basis, Q = H^-1 Qbar H
// (Section 2.2.2); u and out may be the same vector.
ctm_status recombine(ctm_plan* P, const double* u, double* out, hipStream_t s) {
  ctm_status st = ensure_hier(P);
  if (st != CTM_OK) return st;
  CTM_HIP(launch_hierarchize(P->dgrids, P->G, P->maxpts, P->lattice, false, u, out, s));
  CTM_HIP(launch_hier_combine(P->dhoff, P->dhidx, P->dhcoef, P->hnodes, out, P->dhsg, s));
  CTM_HIP(launch_hier_scatter(P->dhnode, P->slen, P->dhsg, out, s));
  CTM_HIP(launch_hierarchize(P->dgrids, P->G, P->maxpts, P->lattice, true, out, out, s));
  return CTM_OK;
}

// MGRIT on one block: X (start) -> Y (state at the block end).
// Level-0 correction of an FCF iteration, per size class on the class's
// lane (after its cycle): U[m] = Un[m] + E[m], m = 1..M0.
ctm_status correct_by_class(ctm_plan* P, double* U, double* Un, double* E, long long M0,
                            hipStream_t s) {
  return class_vec_add(P, vref(U, 1, 1), vref(Un, 1, 1), vref(E, 1, 1), M0, s);
}

ctm_status mgrit_block(ctm_plan* P, Layout& lay, hipStream_t s) {
  const ctm_problem& p = P->prob;
  ctm_status st;
  if (lay.L == 1) {
    ChainArgs a = base_args(P, 0, (int)lay.N[0]);
    a.start = vref(lay.X, 0, 0);
    a.fin = vref(lay.Y, 0, 0);
    TaskSet* single = nullptr;
    if ((st = tasks_for(P, 1, &single)) != CTM_OK) return st;
    return run_chain(P, a, *single, s);
  }
  const long long c = lay.c;
  const long long M0 = lay.N[0] / c;
  TaskSet* tasks = nullptr;
  if ((st = tasks_for(P, M0, &tasks)) != CTM_OK) return st;
  const long long nt = tasks->total;
  const bool fcf = (p.relax == CTM_RELAX_FCF);
  // initial guess: the start state at every C-point
  CTM_HIP(launch_vec_add(vref(lay.U, 1, 0), vref(lay.X, 0, 0), vref(nullptr, 0, 0), (int)(M0 + 1),
                         P->slen, s));
  if (fcf) CTM_HIP(hipMemcpyAsync(lay.Un, lay.X, P->slen * sizeof(double), hipMemcpyDeviceToDevice, s));
  for (int l = 1; l < lay.L; ++l) CTM_HIP(launch_fill_zero(lay.R[l], P->slen, s));  // r_0 = 0
  CTM_HIP(launch_fill_zero(lay.E[lay.L - 1], P->slen, s));  // e_0 = 0 on the last level
  CTM_HIP(launch_grid_norms2(P->dgrids, P->G, lay.X, P->dnorm2, s));
  double* U = lay.U;
  double* Un = lay.Un;
  // warm starts: every relaxation stores its F-points in the trajectory, and
  // once it holds values, each fine solve starts from the value at its own
  // time point (the last step of an interval from the current C-point)
  double* Tr = lay.Tr;
  bool traj = false;
  // The convergence test runs on the device. Iteration it is queued before
  // the host waits for the test of iteration it - 1, so the GPU always has
  // work; once the test stops the block, everything queued after it does
  // nothing (skip), and the C-points keep the stopping iteration's values.
  const int maxit = p.mgrit_maxit;
  CTM_HIP(launch_fill_zero(P->dmg, 2LL * (maxit + 1), s));
  while ((int)P->it_events.size() <= maxit) {
    hipEvent_t e = nullptr;
    CTM_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    P->it_events.push_back(e);
  }
  std::vector<double*> Cit(maxit + 1, nullptr);  // C-point buffer of each iteration
  P->skip = P->dmg;
  struct SkipOff {
    ctm_plan* P;
    ~SkipOff() { P->skip = nullptr; }
  } skip_off{P};
  int stop = 0;      // stopping iteration found by the host (0: none yet)
  int queued = 0;
  // reads the test of iteration k (queued earlier); returns true when the
  // block has stopped at or before k
  // launch bookkeeping after the test of each iteration: launches queued
  // past the stopping iteration do nothing and are taken back out
  struct Mark {
    long long launches;
    double bytes;
    double shape_bytes[16];
    size_t events_used;
  };
  std::vector<Mark> marks(maxit + 1);
  auto mark = [&](int k) {
    Mark& m = marks[k];
    m.launches = P->stats.chain_launches;
    m.bytes = P->stats.chain_bytes;
    std::memcpy(m.shape_bytes, P->stats.shape_bytes, sizeof(m.shape_bytes));
    m.events_used = P->events_used;
  };
  auto rewind = [&](int k) {
    const Mark& m = marks[k];
    P->stats.chain_launches = m.launches;
    P->stats.chain_bytes = m.bytes;
    std::memcpy(P->stats.shape_bytes, m.shape_bytes, sizeof(m.shape_bytes));
    P->events_used = m.events_used;
  };
  auto observe = [&](int k) -> ctm_status {
    if (hipEventSynchronize(P->it_events[k]) != hipSuccess)
      return fail(CTM_ERR_HIP, "hipEventSynchronize failed");
    const double res = P->hmg[2 * k];
    const int at = (int)P->hmg[2 * k + 1];
    if (at == 0 || at == k) {
      P->stats.mgrit_iterations += 1;
      if (P->stats.history_len < CTM_MAX_HISTORY)
        P->stats.mgrit_residual[P->stats.history_len++] = res;
    }
    if (at != 0) stop = at;
    return CTM_OK;
  };
  int seen = 0;  // iterations observed so far
  // FCF: the C-relaxation writes the C-points to Un, and the level-0
  // correction writes u_cm + e_m to U (out of place), from which the next
  // FC-relaxation starts; Un keeps each iteration's C-points as its
  // relaxation left them. Every phase of one class reads only what the same
  // class wrote before, so with per_class the phases, the coarse cycle and
  // the correction follow each other on the class's lane without
  // cross-stream synchronisation; only the convergence test joins all lanes.
  bool open = false;  // side streams hold work not yet joined into s
  // the schedule (CTM_SCHED_AUTO): two levels run every phase per class
  // without joins (measured faster on heat3d); three or more join each phase
  // (measured faster on ou4d, where the slowest class's relaxation then has
  // the machine to itself at the end of each phase instead of sharing it
  // with the next phase of the other classes)
  const bool per_class = P->sched == CTM_SCHED_AUTO ? (lay.L == 2)
                                                     : (P->sched == CTM_SCHED_PER_CLASS);
  for (int it = 1; it <= maxit; ++it) {
    // when the residuals seen so far predict that iteration it - 1 meets the
    // tolerance (geometric decrease), wait for its test before queueing more
    if (it >= 2 && seen == it - 2 && seen >= 2) {
      const double r1 = P->hmg[2 * seen], r0 = P->hmg[2 * (seen - 1)];
      if (r0 > 0 && r1 * (r1 / r0) <= p.mgrit_tol) {
        if ((st = observe(it - 1)) != CTM_OK) return st;
        seen = it - 1;
        if (stop) break;
      }
    }
    double* C;
    if (fcf) {
      ChainArgs fc = base_args(P, 0, (int)c, false, true);
      fc.ftq = (double)c * fc.dt;  // task q starts at fine step c q
      fc.start = vref(U, 1, 0);
      fc.fin = vref(Un, 1, 1);
      if (Tr) {
        fc.inter = vref(Tr, c, 0);
        if (traj) {
          fc.guess = vref(Tr, c, 0);
          fc.guess_fin = vref(U, 1, 1);
        }
      }
      if ((st = run_chain(P, fc, *tasks, s, false, !open, !per_class)) != CTM_OK) return st;
      open = per_class;
      traj = (Tr != nullptr);
      C = Un;
    } else {
      C = U;
    }
    Cit[it] = C;
    ChainArgs fr = base_args(P, 0, (int)c, false, true);
    fr.ftq = (double)c * fr.dt;
    fr.start = vref(C, 1, 0);
    fr.fin = vref(lay.R[1], 1, 1);
    fr.target = vref(C, 1, 1);
    fr.res2 = lay.res2;
    if (Tr) {
      fr.inter = vref(Tr, c, 0);
      if (traj) {
        fr.guess = vref(Tr, c, 0);
        fr.guess_fin = vref(C, 1, 1);
      }
    }
    if ((st = run_chain(P, fr, *tasks, s, false, !open, true)) != CTM_OK) return st;
    open = false;
    traj = (Tr != nullptr);
    CTM_HIP(launch_residual_max(tasks->d, (int)nt, lay.res2, P->dnorm2, lay.rpart, P->dmg,
                                P->hmg_dev, it, p.mgrit_tol,
                                reinterpret_cast<const int*>(P->dsync + 1), s));
    CTM_HIP(hipEventRecord(P->it_events[it], s));
    mark(it);
    queued = it;
    if (it < maxit) {
      if (fcf) {
        if (per_class) {
          // the lanes see the convergence test (its stop flag), then run the
          // coarse chain and the correction class by class
          if ((st = fork_lanes(P, s)) != CTM_OK) return st;
          if ((st = cycle(P, lay, 1, s, true)) != CTM_OK) return st;
          if ((st = correct_by_class(P, U, Un, lay.E[1], M0, s)) != CTM_OK) return st;
          open = true;
        } else {
          if ((st = cycle(P, lay, 1, s, false)) != CTM_OK) return st;
          CTM_HIP(launch_vec_add(vref(U, 1, 1), vref(Un, 1, 1), vref(lay.E[1], 1, 1), (int)M0,
                                 P->slen, s, P->skip));
          open = false;
        }
      } else {
        if ((st = cycle(P, lay, 1, s, false)) != CTM_OK) return st;
        CTM_HIP(launch_vec_add(vref(C, 1, 0), vref(C, 1, 0), vref(lay.E[1], 1, 0),
                               (int)(M0 + 1), P->slen, s, P->skip));
      }
    }
    if (it >= 2 && seen < it - 1) {
      if ((st = observe(it - 1)) != CTM_OK) return st;
      seen = it - 1;
    }
    if (stop) break;
  }
  if (open && (st = join_lanes(P, s)) != CTM_OK) return st;
  if (!stop && seen < queued && (st = observe(queued)) != CTM_OK) return st;
  const int last = stop ? stop : queued;
  if (stop) rewind(stop);
  CTM_HIP(hipMemcpyAsync(lay.Y, Cit[last] + M0 * P->slen, P->slen * sizeof(double),
                         hipMemcpyDeviceToDevice, s));
  if (stop) {
    const double res = P->hmg[2 * stop];
    if (!(res <= p.mgrit_tol)) return fail(CTM_ERR_NONFINITE, "non-finite value in MGRIT");
    return CTM_OK;
  }
  return fail(CTM_ERR_NOCONV, "MGRIT reached mgrit_maxit");
}

// ------------------------------------------------ allocation-free solve
// The workspace of ctm_solve_noalloc: one array in the library's device
// code, CTM_NOALLOC_WORKSPACE_BYTES long, held by every device the library
// runs on until the process ends. Host code never passes its name to a
// kernel or copy (on the host the name is only a stand-in); it uses the
// device address hipGetSymbolAddress returns, one per device, looked up once
// with that device current.
static __device__ __align__(256) unsigned char scratch[CTM_NOALLOC_WORKSPACE_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the array on device dev (the current device), looked up
// on first use; nullptr if the lookup fails.
void* scratch_address(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) == hipSuccess) g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

// Task sets a solve launches: the level-0 intervals, the intervals of every
// intermediate MGRIT level, and one task per grid.
std::vector<long long> solve_task_counts(const ctm_plan* P) {
  const ctm_problem& p = P->prob;
  std::vector<long long> m{1};
  if (p.mgrit_levels > 1) {
    long long n = p.nsteps / p.nrecomb;
    for (int l = 0; l < p.mgrit_levels - 1; ++l) {
      m.push_back(n / p.mgrit_cf);
      n /= p.mgrit_cf;
    }
  }
  return m;
}

constexpr size_t kSyncEvents = 4;  // fork/join events one phase uses at most

// Builds what ctm_solve otherwise creates on first use: the task sets, the
// side streams, the fork/join and per-iteration events, and the node map of
// the hierarchical basis when there are recombination steps.
ctm_status prepare_solve(ctm_plan* P) {
  ctm_status st;
  for (long long M : solve_task_counts(P)) {
    TaskSet* ts = nullptr;
    if ((st = tasks_for(P, M, &ts)) != CTM_OK) return st;
  }
  for (int l = 1; l <= ctm_plan::kSideStreams; ++l) {
    hipStream_t cs = nullptr;
    if ((st = lane_stream(P, l, nullptr, &cs)) != CTM_OK) return st;
  }
  size_t used = 0;
  while (P->sync_events.size() < kSyncEvents)
    if (!take_event(P, used, P->sync_events, false)) return fail(CTM_ERR_HIP, "event creation failed");
  while ((int)P->it_events.size() <= P->prob.mgrit_maxit) {
    hipEvent_t e = nullptr;
    CTM_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    P->it_events.push_back(e);
  }
  if (P->prob.nrecomb > 1 && (st = ensure_hier(P)) != CTM_OK) return st;
  return CTM_OK;
}

// Whether a solve would find everything prepare_solve builds.
bool solve_prepared(const ctm_plan* P) {
  for (long long M : solve_task_counts(P))
    if (!P->tsets.count(M)) return false;
  for (auto s : P->cstreams)
    if (!s) return false;
  if (P->sync_events.size() < kSyncEvents) return false;
  if ((int)P->it_events.size() <= P->prob.mgrit_maxit) return false;
  if (P->prob.nrecomb > 1 && !P->dhnode) return false;
  return true;
}

// The problem's initial value on every grid.
hipError_t initial_state(ctm_plan* P, double* u0, hipStream_t s) {
  if (P->prob.manufactured == CTM_MMS_HEAT)
    return launch_mms_initial(P->dgrids, P->G, P->maxpts, P->prob.t0, u0, s);
  return launch_initial_state(P->dgrids, P->G, P->maxpts, P->n, (int)P->icw.size(), P->dicw,
                              P->dicf, u0, s);
}

// The body of ctm_solve on a given workspace.
ctm_status solve_on(ctm_plan* P, void* ws, size_t ws_bytes, const double* u0, double* u_final,
                    hipStream_t hs) {
  Layout lay = make_layout(P, static_cast<char*>(ws));
  if (ws_bytes < lay.bytes) return fail(CTM_ERR_NOMEM, "workspace smaller than ctm_plan_workspace_bytes");
  reset_stats(P);
  ctm_status st = reset_device_stats(P, hs);
  if (st != CTM_OK) return st;
  if (u0) {
    CTM_HIP(hipMemcpyAsync(lay.X, u0, P->slen * sizeof(double), hipMemcpyDeviceToDevice, hs));
  } else {
    CTM_HIP(initial_state(P, lay.X, hs));
  }
  ctm_status result = CTM_OK;
  const double dt0 = (P->prob.t1 - P->prob.t0) / (double)P->prob.nsteps;
  const long long Nb = P->prob.nsteps / P->prob.nrecomb;
  for (int b = 0; b < P->prob.nrecomb; ++b) {
    if (b > 0 && (st = recombine(P, lay.Y, lay.X, hs)) != CTM_OK) return st;
    P->block_t0 = P->prob.t0 + (double)(b * Nb) * dt0;
    st = mgrit_block(P, lay, hs);
    // the caller's stream waits for the side lanes whatever happened (an
    // error can leave a phase running on them)
    const ctm_status js = join_lanes(P, hs);
    if (st == CTM_OK && js != CTM_OK) st = js;
    P->stats.blocks += 1;
    if (st == CTM_ERR_NOCONV) {
      result = st;
    } else if (st != CTM_OK) {
      return st;
    }
  }
  P->block_t0 = P->prob.t0;
  CTM_HIP(hipMemcpyAsync(u_final, lay.Y, P->slen * sizeof(double), hipMemcpyDeviceToDevice, hs));
  if ((st = collect_device_stats(P, hs)) != CTM_OK) return st;
  if (result != CTM_OK) return result;
  return status_from_flags(P->stats.status_flags);
}

}  // namespace

extern "C" {

const char* ctm_last_error(void) { return g_last_error.c_str(); }

const char* ctm_status_string(ctm_status st) {
  switch (st) {
    case CTM_OK: return "ok";
    case CTM_ERR_INVALID: return "invalid argument";
    case CTM_ERR_NOMEM: return "out of memory";
    case CTM_ERR_HIP: return "HIP error";
    case CTM_ERR_NOCONV: return "no convergence";
    case CTM_ERR_BREAKDOWN: return "Krylov breakdown";
    case CTM_ERR_NONFINITE: return "non-finite value";
  }
  return "unknown status";
}

ctm_status ctm_problem_defaults(ctm_problem* p) {
  if (!p) return fail(CTM_ERR_INVALID, "problem is NULL");
  std::memset(p, 0, sizeof(*p));
  p->d = 2;
  p->level_n = 4;
  p->level_min = 1;
  for (int i = 0; i < CTM_MAXD; ++i) {
    p->lo[i] = 0.0;
    p->hi[i] = 1.0;
  }
  p->op = CTM_OP_HEAT;
  p->t0 = 0.0;
  p->t1 = 1.0;
  p->nsteps = 16;
  p->nrecomb = 1;
  p->mgrit_levels = 2;
  p->mgrit_cf = 2;
  p->relax = CTM_RELAX_FCF;
  p->mgrit_tol = 1e-8;
  p->mgrit_maxit = 100;
  p->krylov = CTM_KRYLOV_AUTO;
  p->krylov_tol = 1e-8;
  p->krylov_maxit = 10000;
  p->prec = CTM_PREC_FP64;
  p->refine_tol = 1e-8;
  p->inner_tol = 1e-5;
  p->refine_maxit = 10;
  p->warm_start = 1;
  p->precond = CTM_PRECOND_LINE;
  p->schwarz_s = 5;
  return CTM_OK;
}

ctm_status ctm_plan_create(const ctm_problem* prob, ctm_plan** out) {
  if (!out) return fail(CTM_ERR_INVALID, "plan output pointer is NULL");
  *out = nullptr;
  ctm_status st = validate(prob);
  if (st != CTM_OK) return st;
  ctm_plan* P = new (std::nothrow) ctm_plan();
  if (!P) return fail(CTM_ERR_NOMEM, "host allocation failed");
  P->prob = *prob;
  P->block_t0 = prob->t0;
  P->d = prob->d;
  P->n = prob->level_n;
  const int F = (1 << P->n) + 1;
  if (prob->ic_terms > 0) {
    P->icw.assign(prob->ic_weight, prob->ic_weight + prob->ic_terms);
    P->icf.assign(prob->ic_factor, prob->ic_factor + (size_t)prob->ic_terms * P->d * F);
  } else {  // manufactured problem without tables: one zero term keeps the buffers valid
    P->icw.assign(1, 0.0);
    P->icf.assign((size_t)P->d * F, 0.0);
  }
  P->prob.ic_weight = nullptr;
  P->prob.ic_factor = nullptr;
  P->lattice = (prob->op == CTM_OP_CME);
  P->opc = prob->op == CTM_OP_HEAT      ? OPC_HEAT
           : prob->op == CTM_OP_VARCOEF ? OPC_VAR
           : prob->op == CTM_OP_DRIFT   ? OPC_DRIFT
                                        : OPC_SEP;
  const bool sym = (prob->op == CTM_OP_HEAT || prob->op == CTM_OP_VARCOEF);
  P->solver = (prob->krylov == CTM_KRYLOV_BICGSTAB || (prob->krylov == CTM_KRYLOV_AUTO && !sym))
                  ? SOLV_BICG : SOLV_CG;
  P->mixed = (prob->prec == CTM_PREC_MIXED);
  hipGetDevice(&P->device);

  // combination index set: layer w ascending, l lexicographic
  const int d = P->d;
  long long off = 0;
  for (int w = 0; w < d; ++w) {
    const int total = P->n + d - 1 - w;
    if (total < d * prob->level_min) continue;
    std::vector<std::vector<int>> ls;
    std::vector<int> cur;
    compositions(total, d, prob->level_min, cur, ls);
    const double coef = ((w & 1) ? -1.0 : 1.0) * (double)binom(d - 1, w);
    for (auto& l : ls) {
      GridHost gh;
      std::memset(&gh, 0, sizeof(gh));
      long long np = 1;
      for (int i = 0; i < d; ++i) {
        gh.lev[i] = l[i];
        np *= P->lattice ? (1LL << l[i]) : ((1LL << l[i]) - 1);
      }
      gh.w = w;
      gh.coef = coef;
      gh.npts = np;
      gh.off = off;
      off += np;
      P->grids.push_back(gh);
    }
  }
  P->G = (int)P->grids.size();
  P->slen = off;
  if (P->G > 65535) {  // per-grid kernels index grids by the launch grid's y extent
    delete P;
    return fail(CTM_ERR_INVALID, "more than 65,535 component grids");
  }
  for (auto& gh : P->grids) P->maxpts = (int)std::max<long long>(P->maxpts, gh.npts);
  if (P->maxpts > (1 << 20)) {
    delete P;
    return fail(CTM_ERR_INVALID, "a component grid has more than 2^20 unknowns");
  }

  const double dt0 = (prob->t1 - prob->t0) / (double)prob->nsteps;
  for (auto& gh : P->grids) {
    GridDev gd;
    std::memset(&gd, 0, sizeof(gd));
    gd.npts = (int)gh.npts;
    gd.d = d;
    gd.off = gh.off;
    gd.j0 = P->lattice ? 0 : 1;
    gd.coef = gh.coef;
    long long stride = 1;
    for (int i = d - 1; i >= 0; --i) {
      gd.lev[i] = gh.lev[i];
      gd.n[i] = P->lattice ? (1 << gh.lev[i]) : ((1 << gh.lev[i]) - 1);
      gd.stride[i] = (int)stride;
      gd.cstride[i] = (int)stride;
      stride *= gd.n[i];
      gd.lo[i] = prob->lo[i];
      gd.h[i] = (prob->hi[i] - prob->lo[i]) / (double)(1LL << gh.lev[i]);
      gd.ih2[i] = 1.0 / (gd.h[i] * gd.h[i]);
    }
    build_tables(P, gh, gd);
    P->tabmax = std::max(P->tabmax, gd.tabsz);
    // stiff axis: strongest coupling (largest off-diagonal magnitude of L
    // along the axis); ties go to the longer axis, then the lower index
    double best = -1.0;
    int sax = 0;
    for (int i = 0; i < d; ++i) {
      double strength = 0.0;
      if (P->opc == OPC_SEP) {
        const double* t = P->htab.data() + gd.tab0 + gd.tab[i];
        for (int j = 0; j < gd.n[i]; ++j)
          strength = std::max(strength, std::fabs(t[j]) + std::fabs(t[2 * gd.n[i] + j]));
      } else if (P->opc == OPC_DRIFT) {
        // diffusion plus the largest face velocity over the box
        double wmax = 0.0;
        for (int c2 = 0; c2 < d; ++c2)
          wmax += std::fabs(prob->drift[i * d + c2]) *
                  std::max(std::fabs(prob->lo[c2]), std::fabs(prob->hi[c2]));
        strength = prob->diffusion[i] * gd.ih2[i] + wmax / gd.h[i];
      } else {
        strength = gd.ih2[i];
      }
      if (gd.n[i] == 1) strength = 0.0;  // nothing to couple along this axis
      if (strength > best * (1 + 1e-12) ||
          (std::fabs(strength - best) <= 1e-12 * best && gd.n[i] > gd.n[sax])) {
        best = strength;
        sax = i;
      }
    }
    gd.sax = sax;
    gd.ns = gd.n[sax];
    gd.nlines = gd.npts / gd.ns;
    gd.nseg = (gd.ns + kSegLen - 1) / kSegLen;
    int m = 0;
    for (int i = 0; i < d; ++i)
      if (i != sax) gd.oax[m++] = i;
    int ls = 1;
    for (int mm = d - 2; mm >= 0; --mm) {
      gd.lstride[mm] = ls;
      ls *= gd.n[gd.oax[mm]];
    }
    // cost estimate for longest-first scheduling: unknowns * sqrt(condition)
    double lam = 0.0;
    for (int i = 0; i < d; ++i) lam += 4.0 * gd.ih2[i];
    gh.cost = (double)gh.npts * std::sqrt(1.0 + dt0 * lam);
    P->hdev.push_back(gd);
  }
  // grids the on-chip shapes cannot hold go to the streaming kernel
  P->shape = pick_shape(P->hdev);
  P->gshape.resize(P->G);
  int nstream = 0, maxstream = 0;
  P->schwarz = (prob->precond == CTM_PRECOND_SCHWARZ);
  for (int g = 0; g < P->G; ++g) {
    // the Schwarz preconditioner lives in the streaming solver only
    const int sh = P->schwarz ? -1 : grid_shape_fitting(P, P->hdev[g]);
    P->gshape[g] = sh >= 0 ? sh : kStreamShape;
    if (sh < 0) {
      ++nstream;
      maxstream = std::max(maxstream, P->hdev[g].npts);
      // (lines longer than kSegLen unknowns: the line preconditioner
      // works on segments of them)
    }
  }
  if (nstream) {
    if ((size_t)P->tabmax * sizeof(double) > 65536) {
      delete P;
      return fail(CTM_ERR_INVALID, "coefficient tables of a streaming grid exceed 64 KiB");
    }
    // scratch for the largest launch: every streaming grid times the
    // level-0 intervals of a block (or one task per grid)
    const long long nb = prob->nsteps / prob->nrecomb;
    const long long M = (prob->mgrit_levels > 1) ? std::max<long long>(1, nb / prob->mgrit_cf) : 1;
    P->stream_ss = ((long long)maxstream + 63) / 64 * 64;
    P->stream_tasks = (long long)nstream * M;
    // work-groups per task of the wide solver, for the largest grid
    for (int g = 0; g < P->G; ++g) {
      if (P->gshape[g] != kStreamShape) continue;
      const GridDev& gd = P->hdev[g];
      const int seglen = gd.nseg > 1 ? kSegLen : gd.ns;
      int Lc = 1;
      while (Lc < (seglen + kWideSK - 1) / kWideSK) Lc <<= 1;
      const int waves = (gd.nlines * gd.nseg + 64 / Lc - 1) / (64 / Lc);
      P->wide_lb = std::max(P->wide_lb, (waves + kWLW - 1) / kWLW);
      P->wide_pb = std::max(P->wide_pb, (gd.npts + kWP - 1) / kWP);
    }
    P->wide_maxblk = std::max(P->wide_pb, P->wide_lb);
  }
  assign_lanes(P);
  if (P->htab.empty()) P->htab.push_back(0.0);
  P->order.resize(P->G);
  for (int g = 0; g < P->G; ++g) P->order[g] = g;
  std::stable_sort(P->order.begin(), P->order.end(),
                   [&](int a, int b) { return P->grids[a].cost > P->grids[b].cost; });

  auto cleanup = [&](ctm_status s2) {
    delete P;
    return s2;
  };
#define CTM_HIPC(call)                                                                     \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return cleanup(fail(CTM_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_))); \
  } while (0)
  CTM_HIPC(hipMalloc(&P->dgrids, P->G * sizeof(GridDev)));
  CTM_HIPC(hipMemcpy(P->dgrids, P->hdev.data(), P->G * sizeof(GridDev), hipMemcpyHostToDevice));
  CTM_HIPC(hipMalloc(&P->dtab, P->htab.size() * sizeof(double)));
  CTM_HIPC(hipMemcpy(P->dtab, P->htab.data(), P->htab.size() * sizeof(double), hipMemcpyHostToDevice));
  std::vector<long long> offs(P->G);
  for (int g = 0; g < P->G; ++g) offs[g] = P->grids[g].off;
  CTM_HIPC(hipMalloc(&P->doffsets, P->G * sizeof(long long)));
  CTM_HIPC(hipMemcpy(P->doffsets, offs.data(), P->G * sizeof(long long), hipMemcpyHostToDevice));
  CTM_HIPC(hipMalloc(&P->dicw, P->icw.size() * sizeof(double)));
  CTM_HIPC(hipMemcpy(P->dicw, P->icw.data(), P->icw.size() * sizeof(double), hipMemcpyHostToDevice));
  CTM_HIPC(hipMalloc(&P->dicf, P->icf.size() * sizeof(double)));
  CTM_HIPC(hipMemcpy(P->dicf, P->icf.data(), P->icf.size() * sizeof(double), hipMemcpyHostToDevice));
  CTM_HIPC(hipMalloc(&P->dcounters, kStatSlots * CNT_N * sizeof(unsigned long long)));
  CTM_HIPC(hipMemset(P->dcounters, 0, kStatSlots * CNT_N * sizeof(unsigned long long)));
  CTM_HIPC(hipMalloc(&P->dsync, 2 * sizeof(double)));
  CTM_HIPC(hipMemset(P->dsync, 0, 2 * sizeof(double)));
  CTM_HIPC(hipMalloc(&P->dnorm2, P->G * sizeof(double)));
  CTM_HIPC(hipHostMalloc(&P->hsync, 2 * sizeof(double), hipHostMallocDefault));
  if (P->stream_tasks) {
    const size_t bytes =
        (size_t)P->stream_tasks * kStreamVectors * (size_t)P->stream_ss * sizeof(double);
    if (hipMalloc(&P->dstream, bytes) != hipSuccess)
      return cleanup(fail(CTM_ERR_NOMEM, "streaming scratch allocation failed"));
    const int cap = (int)std::min<long long>(P->stream_tasks, ctm_plan::kWideMaxGridY);
    P->wide_cap = cap;
    CTM_HIPC(hipMalloc(&P->dwide, cap * sizeof(WideTask)));
    CTM_HIPC(hipMemset(P->dwide, 0, cap * sizeof(WideTask)));
    CTM_HIPC(hipMalloc(&P->dwpart, (size_t)cap * WS_N * P->wide_maxblk * sizeof(double)));
    CTM_HIPC(hipHostMalloc(&P->hwide, cap * sizeof(int),
                           hipHostMallocMapped | hipHostMallocCoherent));
    std::memset(P->hwide, 0, cap * sizeof(int));
    CTM_HIPC(hipHostGetDevicePointer(reinterpret_cast<void**>(&P->hwide_dev), P->hwide, 0));
    CTM_HIPC(hipEventCreateWithFlags(&P->wide_ev, hipEventDisableTiming));
  }
  {
    const size_t nmg = 2 * (size_t)(std::max(1, prob->mgrit_maxit) + 1);
    CTM_HIPC(hipMalloc(&P->dmg, nmg * sizeof(double)));
    CTM_HIPC(hipHostMalloc(&P->hmg, nmg * sizeof(double),
                           hipHostMallocMapped | hipHostMallocCoherent));
    std::memset(P->hmg, 0, nmg * sizeof(double));
    CTM_HIPC(hipHostGetDevicePointer(reinterpret_cast<void**>(&P->hmg_dev), P->hmg, 0));
  }
  std::vector<int2> ident(P->G);
  for (int g = 0; g < P->G; ++g) ident[g] = make_int2(g, 0);
  CTM_HIPC(hipMalloc(&P->didentity, P->G * sizeof(int2)));
  CTM_HIPC(hipMemcpy(P->didentity, ident.data(), P->G * sizeof(int2), hipMemcpyHostToDevice));
  {
    // gather stages: runs of consecutive grids, contiguous in the packed
    // vector, whose unknowns fit one LDS stage (a larger grid alone)
    std::vector<int2> st;
    const long long cap = gather_stage_capacity();
    for (int g = 0; g < P->G;) {
      long long n = 0;
      int e = g;
      while (e < P->G && n + P->hdev[e].npts <= cap &&
             (e == g || P->hdev[e].off == P->hdev[e - 1].off + P->hdev[e - 1].npts))
        n += P->hdev[e++].npts;
      if (e == g) e = g + 1;
      st.push_back(make_int2(g, e));
      g = e;
    }
    P->ngstage = (int)st.size();
    CTM_HIPC(hipMalloc(&P->dgstage, st.size() * sizeof(int2)));
    CTM_HIPC(hipMemcpy(P->dgstage, st.data(), st.size() * sizeof(int2), hipMemcpyHostToDevice));
  }
  if (P->schwarz) {
    std::vector<SchwarzGrid> sgs(P->G);
    std::vector<SchwarzSub> subs;
    std::vector<int> ints, subgrid;
    long long linv_len = 0, cinv_len = 0;
    for (int g = 0; g < P->G; ++g) {
      std::string msg;
      std::memset(&sgs[g], 0, sizeof(SchwarzGrid));
      if (!schwarz_decompose(P->hdev[g], prob->schwarz_s, sgs[g], subs, ints, linv_len, cinv_len,
                             msg))
        return cleanup(fail(CTM_ERR_INVALID, msg));
      subgrid.resize(subs.size(), g);
      P->sch_nmax = std::max(P->sch_nmax, sgs[g].nmax);
      P->sch_nbmax = std::max(P->sch_nbmax, sgs[g].nblk);
    }
    P->sch_nsub = (long long)subs.size();
    CTM_HIPC(hipMalloc(&P->dsch_grid, P->G * sizeof(SchwarzGrid)));
    CTM_HIPC(hipMemcpy(P->dsch_grid, sgs.data(), P->G * sizeof(SchwarzGrid),
                       hipMemcpyHostToDevice));
    CTM_HIPC(hipMalloc(&P->dsch_sub, subs.size() * sizeof(SchwarzSub)));
    CTM_HIPC(hipMemcpy(P->dsch_sub, subs.data(), subs.size() * sizeof(SchwarzSub),
                       hipMemcpyHostToDevice));
    CTM_HIPC(hipMalloc(&P->dsch_ints, ints.size() * sizeof(int)));
    CTM_HIPC(hipMemcpy(P->dsch_ints, ints.data(), ints.size() * sizeof(int),
                       hipMemcpyHostToDevice));
    CTM_HIPC(hipMalloc(&P->dsch_subgrid, subgrid.size() * sizeof(int)));
    CTM_HIPC(hipMemcpy(P->dsch_subgrid, subgrid.data(), subgrid.size() * sizeof(int),
                       hipMemcpyHostToDevice));
    // the inverses of every MGRIT level (step dt c^level)
    const int levels = std::max(1, prob->mgrit_levels);
    int* dstat = reinterpret_cast<int*>(P->dsync + 1);
    for (int l = 0; l < levels; ++l) {
      double* li = nullptr;
      double* ci = nullptr;
      if (hipMalloc(&li, std::max<long long>(1, linv_len) * sizeof(double)) != hipSuccess ||
          hipMalloc(&ci, std::max<long long>(1, cinv_len) * sizeof(double)) != hipSuccess) {
        hipFree(li);
        hipFree(ci);
        return cleanup(fail(CTM_ERR_NOMEM, "Schwarz preconditioner allocation failed"));
      }
      P->dsch_linv.push_back(li);
      P->dsch_cinv.push_back(ci);
      const SchwarzView v = schwarz_view(P, l);
      CTM_HIPC(launch_schwarz_setup(P->opc, P->d, P->dgrids, P->G, P->dtab, prob->amp,
                                    level_dt(P, l), P->tabmax, v, li, ci, P->dsch_subgrid,
                                    P->sch_nsub, P->sch_nmax, dstat, nullptr));
    }
    CTM_HIPC(hipDeviceSynchronize());
    int flags = 0;
    CTM_HIPC(hipMemcpy(&flags, dstat, sizeof(int), hipMemcpyDeviceToHost));
    if (flags) return cleanup(fail(CTM_ERR_BREAKDOWN, "Schwarz preconditioner: singular "
                                                      "subdomain or coarse matrix"));
  }
#undef CTM_HIPC
  reset_stats(P);
  if ((st = prepare_solve(P)) != CTM_OK) {
    delete P;
    return st;
  }
  scratch_address(P->device);  // set-up of the allocation-free entry point
  *out = P;
  return CTM_OK;
}

void ctm_plan_destroy(ctm_plan* plan) { delete plan; }

ctm_status ctm_plan_grids(const ctm_plan* P, int* G) {
  if (!P || !G) return fail(CTM_ERR_INVALID, "NULL argument");
  *G = P->G;
  return CTM_OK;
}

ctm_status ctm_plan_grid_info(const ctm_plan* P, int g, int* levels, double* coef,
                              long long* offset, long long* npoints) {
  if (!P) return fail(CTM_ERR_INVALID, "plan is NULL");
  if (g < 0 || g >= P->G) return fail(CTM_ERR_INVALID, "grid index out of range");
  const GridHost& gh = P->grids[g];
  if (levels)
    for (int i = 0; i < P->d; ++i) levels[i] = gh.lev[i];
  if (coef) *coef = gh.coef;
  if (offset) *offset = gh.off;
  if (npoints) *npoints = gh.npts;
  return CTM_OK;
}

ctm_status ctm_plan_state_len(const ctm_plan* P, long long* len) {
  if (!P || !len) return fail(CTM_ERR_INVALID, "NULL argument");
  *len = P->slen;
  return CTM_OK;
}

ctm_status ctm_plan_workspace_bytes(const ctm_plan* P, size_t* bytes) {
  if (!P || !bytes) return fail(CTM_ERR_INVALID, "NULL argument");
  *bytes = make_layout(P, nullptr).bytes;
  return CTM_OK;
}


ctm_status ctm_initial_state(ctm_plan* P, double* u0, ctm_stream s) {
  if (!P || !u0) return fail(CTM_ERR_INVALID, "NULL argument");
  CTM_HIP(initial_state(P, u0, (hipStream_t)s));
  return CTM_OK;
}

ctm_status ctm_apply(ctm_plan* P, int level, const double* x, double* y, ctm_stream s) {
  if (!P || !x || !y) return fail(CTM_ERR_INVALID, "NULL argument");
  if (level < 0 || level > 16) return fail(CTM_ERR_INVALID, "level out of range");
  if (x == y) return fail(CTM_ERR_INVALID, "x and y must not overlap");
  if (P->shape < 0)  // some grid streams: the point-wise apply for every grid
    CTM_HIP(launch_stream_apply(P->opc, P->d, P->dgrids, P->G, P->dtab, P->prob.amp,
                                level_dt(P, level), P->tabmax, x, y, (hipStream_t)s));
  else
    CTM_HIP(launch_apply(P->opc, P->shape, P->dgrids, P->G, P->dtab, P->prob.amp,
                         level_dt(P, level), P->tabmax, x, y, (hipStream_t)s));
  return CTM_OK;
}

ctm_status ctm_precond_apply(ctm_plan* P, int level, const double* x, double* y,
                             ctm_stream s) {
  if (!P || !x || !y) return fail(CTM_ERR_INVALID, "NULL argument");
  if (!P->schwarz) return fail(CTM_ERR_INVALID, "the plan has no Schwarz preconditioner");
  if (level < 0 || level >= (int)P->dsch_linv.size())
    return fail(CTM_ERR_INVALID, "level out of range (the plan's MGRIT levels)");
  if (x == y) return fail(CTM_ERR_INVALID, "x and y must not overlap");
  hipStream_t hs = (hipStream_t)s;
  const long long ss = ((long long)P->maxpts + 63) / 64 * 64;
  double* scratch = nullptr;
  if (hipMalloc(&scratch, (size_t)P->G * kStreamVectors * (size_t)ss * sizeof(double)) !=
      hipSuccess)
    return fail(CTM_ERR_NOMEM, "preconditioner scratch allocation failed");
  hipError_t e = launch_schwarz_apply(P->opc, P->solver, P->d, P->dgrids, P->G, P->dtab,
                                      P->prob.amp, level_dt(P, level), P->tabmax,
                                      schwarz_view(P, level), x, y, scratch, ss, hs);
  if (e == hipSuccess) e = hipStreamSynchronize(hs);
  hipFree(scratch);
  if (e != hipSuccess) return fail(CTM_ERR_HIP, std::string("preconditioner: ") + hipGetErrorString(e));
  return CTM_OK;
}

ctm_status ctm_propagate(ctm_plan* P, int level, long long nsteps, const double* x, double* y,
                         int per_grid, ctm_stream s) {
  if (!P || !x || !y) return fail(CTM_ERR_INVALID, "NULL argument");
  if (level < 0 || level > 16 || nsteps < 0 || nsteps > (1LL << 30))
    return fail(CTM_ERR_INVALID, "level or nsteps out of range");
  if (P->schwarz && level >= (int)P->dsch_linv.size())
    return fail(CTM_ERR_INVALID, "the Schwarz preconditioner is built for the plan's MGRIT levels");
  hipStream_t hs = (hipStream_t)s;
  reset_stats(P);
  ctm_status st = reset_device_stats(P, hs);
  if (st != CTM_OK) return st;
  if (nsteps == 0) {
    if (x != y) CTM_HIP(hipMemcpyAsync(y, x, P->slen * sizeof(double), hipMemcpyDeviceToDevice, hs));
    return CTM_OK;
  }
  if (!per_grid) {
    ChainArgs a = base_args(P, level, (int)nsteps);
    a.start = vref(const_cast<double*>(x), 0, 0);
    a.fin = vref(y, 0, 0);
    TaskSet* single = nullptr;
    if ((st = tasks_for(P, 1, &single)) != CTM_OK) return st;
    return run_chain(P, a, *single, hs);
  }
  for (int g = 0; g < P->G; ++g) {
    for (long long nn = 0; nn < nsteps; ++nn) {
      ChainArgs a = base_args(P, level, 1, true);
      a.start = vref(const_cast<double*>(nn == 0 ? x : y), 0, 0);
      a.fin = vref(y, 0, 0);
      if ((st = run_chain_grid(P, a, g, hs)) != CTM_OK) return st;
    }
  }
  return CTM_OK;
}

ctm_status ctm_solve(ctm_plan* P, void* ws, size_t ws_bytes, const double* u0, double* u_final,
                     ctm_stream s) {
  if (!P || !ws || !u_final) return fail(CTM_ERR_INVALID, "NULL argument");
  return solve_on(P, ws, ws_bytes, u0, u_final, (hipStream_t)s);
}

ctm_status ctm_solve_noalloc(ctm_plan* P, const double* u0, double* u_final, ctm_stream s) {
  if (!P || !u_final) return fail(CTM_ERR_INVALID, "NULL argument");
  const size_t need = make_layout(P, nullptr).bytes;
  if (need > (size_t)CTM_NOALLOC_WORKSPACE_BYTES)
    return fail(CTM_ERR_INVALID, "the plan's workspace (" + std::to_string(need) +
                                     " bytes) exceeds the library's static one (" +
                                     std::to_string((size_t)CTM_NOALLOC_WORKSPACE_BYTES) + " bytes)");
  if (!solve_prepared(P))
    return fail(CTM_ERR_INVALID,
                "the plan's launch tables changed since its last allocating call "
                "(ctm_plan_set_grid_shape, ctm_autotune): call ctm_solve once first");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != P->device)
    return fail(CTM_ERR_INVALID, "the plan's device is not the current device");
  void* ws = scratch_address(P->device);
  if (!ws) return fail(CTM_ERR_HIP, "the static workspace has no device address on this device");
  // per-launch timing would create events: off for this call
  struct TimingOff {
    ctm_plan* P;
    bool was;
    ~TimingOff() { P->timing = was; }
  } timing_off{P, P->timing};
  P->timing = false;
  return solve_on(P, ws, need, u0, u_final, (hipStream_t)s);
}

ctm_status ctm_gather(ctm_plan* P, const double* u, const double* pts, long long npts, double* out,
                      ctm_stream s) {
  if (!P || !u || (!pts && npts > 0) || (!out && npts > 0)) return fail(CTM_ERR_INVALID, "NULL argument");
  if (npts < 0) return fail(CTM_ERR_INVALID, "npts must be >= 0");
  CTM_HIP(launch_gather(P->dgrids, P->dgstage, P->ngstage, P->d, u, pts, npts, out,
                        (hipStream_t)s));
  return CTM_OK;
}

ctm_status ctm_combine_project(ctm_plan* P, const double* u, double* out, ctm_stream s) {
  if (!P || !u || !out) return fail(CTM_ERR_INVALID, "NULL argument");
  if (u == out) return fail(CTM_ERR_INVALID, "u and out must not overlap");
  CTM_HIP(launch_project(P->dgrids, P->doffsets, P->G, P->slen, u, out, (hipStream_t)s));
  return CTM_OK;
}

ctm_status ctm_hierarchize(ctm_plan* P, const double* in, double* out, int inverse,
                           ctm_stream s) {
  if (!P || !in || !out) return fail(CTM_ERR_INVALID, "NULL argument");
  CTM_HIP(launch_hierarchize(P->dgrids, P->G, P->maxpts, P->lattice, inverse != 0, in, out,
                             (hipStream_t)s));
  return CTM_OK;
}

ctm_status ctm_recombine(ctm_plan* P, const double* u, double* out, ctm_stream s) {
  if (!P || !u || !out) return fail(CTM_ERR_INVALID, "NULL argument");
  return recombine(P, u, out, (hipStream_t)s);
}

ctm_status ctm_plan_grid_shape(const ctm_plan* P, int g, int* waves, int* per_lane) {
  if (!P) return fail(CTM_ERR_INVALID, "plan is NULL");
  if (g < 0 || g >= P->G) return fail(CTM_ERR_INVALID, "grid index out of range");
  const int sh = P->gshape[g];
  if (waves) *waves = (sh == kStreamShape) ? 16 : kShapes[sh].W;
  if (per_lane) *per_lane = (sh == kStreamShape) ? 0 : kShapes[sh].K;
  return CTM_OK;
}

ctm_status ctm_plan_set_grid_shape(ctm_plan* P, int g, int waves, int per_lane) {
  if (!P) return fail(CTM_ERR_INVALID, "plan is NULL");
  if (g < 0 || g >= P->G) return fail(CTM_ERR_INVALID, "grid index out of range");
  if (P->gshape[g] == kStreamShape)
    return fail(CTM_ERR_INVALID, "the grid is on the streaming solver");
  int sh = -1;
  for (int s2 = 0; s2 < kNumShapes; ++s2)
    if (kShapes[s2].W == waves && kShapes[s2].K == per_lane) sh = s2;
  if (sh < 0) return fail(CTM_ERR_INVALID, "no such launch shape");
  const GridDev& gd = P->hdev[g];
  if (gd.ns > 64 * per_lane || lanes_needed(gd, per_lane) > 64 * waves)
    return fail(CTM_ERR_INVALID, "the launch shape cannot hold the grid's lines");
  if (!shape_fits(P, gd, sh))
    return fail(CTM_ERR_INVALID, "the launch shape's LDS would exceed a compute unit's");
  set_shape(P, g, sh);
  return CTM_OK;
}

ctm_status ctm_plan_set_wide(ctm_plan* P, int max_tasks) {
  if (!P) return fail(CTM_ERR_INVALID, "plan is NULL");
  if (max_tasks < 0) return fail(CTM_ERR_INVALID, "max_tasks must be >= 0");
  P->wide_max_tasks = std::min(max_tasks, ctm_plan::kWideMaxGridY);
  return CTM_OK;
}

ctm_status ctm_plan_set_schedule(ctm_plan* P, int schedule) {
  if (!P) return fail(CTM_ERR_INVALID, "plan is NULL");
  if (schedule != CTM_SCHED_AUTO && schedule != CTM_SCHED_JOINED &&
      schedule != CTM_SCHED_PER_CLASS)
    return fail(CTM_ERR_INVALID, "unknown schedule");
  P->sched = schedule;
  return CTM_OK;
}

ctm_status ctm_autotune(ctm_plan* P, void* ws, size_t ws_bytes, double* u_scratch,
                        int trial_iterations, int repeats, ctm_tune_report* report,
                        ctm_stream s) {
  if (!P || !ws || !u_scratch) return fail(CTM_ERR_INVALID, "NULL argument");
  if (repeats < 1 || trial_iterations < 0)
    return fail(CTM_ERR_INVALID, "repeats must be >= 1 and trial_iterations >= 0");
  using clock = std::chrono::steady_clock;
  const auto t_start = clock::now();
  hipStream_t hs = (hipStream_t)s;
  // anisotropy classes: grids with equal line length and line count
  struct TuneClass {
    std::vector<int> grids;
    double points = 0.0;
    int cand[2] = {-1, -1};
  };
  std::map<std::pair<int, int>, TuneClass> by_key;
  for (int g = 0; g < P->G; ++g) {
    if (P->gshape[g] == kStreamShape) continue;
    const GridDev& gd = P->hdev[g];
    TuneClass& tc = by_key[{gd.ns, gd.nlines}];
    tc.grids.push_back(g);
    tc.points += (double)gd.npts;
    const int c4 = min_waves_shape(gd, 4), c8 = min_waves_shape(gd, 8);
    tc.cand[0] = (c4 >= 0 && shape_fits(P, gd, c4)) ? c4 : -1;
    tc.cand[1] = (c8 >= 0 && shape_fits(P, gd, c8)) ? c8 : -1;
  }
  std::vector<TuneClass> classes;
  for (auto& kv : by_key)
    if (kv.second.cand[0] >= 0 && kv.second.cand[1] >= 0) classes.push_back(kv.second);
  std::stable_sort(classes.begin(), classes.end(),
                   [](const TuneClass& a, const TuneClass& b) { return a.points > b.points; });
  const std::vector<int> initial = P->gshape;
  const bool timing = P->timing;
  const int maxit = P->prob.mgrit_maxit;
  P->timing = false;
  if (trial_iterations > 0 && P->prob.mgrit_levels > 1)
    P->prob.mgrit_maxit = std::min(maxit, trial_iterations);
  ctm_tune_report rep{};
  rep.classes = (int)classes.size();
  // fastest of `repeats` trial solves with the current shapes
  auto trial = [&](double* best) -> ctm_status {
    *best = 1e300;
    for (int r = 0; r < repeats; ++r) {
      if (hipStreamSynchronize(hs) != hipSuccess)
        return fail(CTM_ERR_HIP, "hipStreamSynchronize failed");
      const auto t0 = clock::now();
      ctm_status st = ctm_solve(P, ws, ws_bytes, nullptr, u_scratch, s);
      if (hipStreamSynchronize(hs) != hipSuccess)
        return fail(CTM_ERR_HIP, "hipStreamSynchronize failed");
      const double ms = std::chrono::duration<double, std::milli>(clock::now() - t0).count();
      rep.trials += 1;
      if (st != CTM_OK && st != CTM_ERR_NOCONV) return st;
      *best = std::min(*best, ms);
    }
    return CTM_OK;
  };
  double cur = 0.0;
  ctm_status st = trial(&cur);
  rep.ms_default = cur;
  for (size_t i = 0; st == CTM_OK && i < classes.size(); ++i) {
    const TuneClass& tc = classes[i];
    const int now = P->gshape[tc.grids[0]];
    const int alt = (now == tc.cand[0]) ? tc.cand[1] : tc.cand[0];
    for (int g : tc.grids) set_shape(P, g, alt);
    double t = 0.0;
    st = trial(&t);
    if (st == CTM_OK && t < 0.98 * cur) {
      cur = t;
    } else {
      for (int g : tc.grids) set_shape(P, g, now);
    }
  }
  // the schedule: the explicit one not in effect, kept on the same rule
  const int sched0 = P->sched;
  if (st == CTM_OK && P->prob.mgrit_levels > 1 && P->prob.relax == CTM_RELAX_FCF) {
    const bool pc_now = (sched0 == CTM_SCHED_AUTO) ? (P->prob.mgrit_levels == 2)
                                                    : (sched0 == CTM_SCHED_PER_CLASS);
    P->sched = pc_now ? CTM_SCHED_JOINED : CTM_SCHED_PER_CLASS;
    double t = 0.0;
    st = trial(&t);
    if (st == CTM_OK && t < 0.98 * cur) {
      cur = t;
    } else {
      P->sched = sched0;
    }
  }
  P->timing = timing;
  P->prob.mgrit_maxit = maxit;
  if (st != CTM_OK) {
    for (int g = 0; g < P->G; ++g) set_shape(P, g, initial[g]);
    P->sched = sched0;
    return st;
  }
  rep.ms_tuned = cur;
  rep.schedule = P->sched;
  for (const TuneClass& tc : classes)
    if (P->gshape[tc.grids[0]] != initial[tc.grids[0]]) rep.changed += 1;
  rep.tune_ms = std::chrono::duration<double, std::milli>(clock::now() - t_start).count();
  if (report) *report = rep;
  return CTM_OK;
}

ctm_status ctm_set_timing(ctm_plan* P, int on) {
  if (!P) return fail(CTM_ERR_INVALID, "plan is NULL");
  P->timing = (on != 0);
  P->events_used = 0;
  return CTM_OK;
}

ctm_status ctm_get_stats(const ctm_plan* Pc, ctm_stats* st) {
  if (!Pc || !st) return fail(CTM_ERR_INVALID, "NULL argument");
  ctm_plan* P = const_cast<ctm_plan*>(Pc);
  if (P->events_used) {
    ctm_status s2 = accumulate_timing(P);
    if (s2 != CTM_OK) return s2;
  }
  // counters live on the device; the caller has synchronised its stream
  unsigned long long c[kStatSlots * CNT_N];
  int flags = 0;
  CTM_HIP(hipMemcpy(c, P->dcounters, sizeof(c), hipMemcpyDeviceToHost));
  CTM_HIP(hipMemcpy(&flags, P->dsync + 1, sizeof(int), hipMemcpyDeviceToHost));
  *st = P->stats;
  fold_counters(P, c, st);
  st->status_flags = flags;
  return CTM_OK;
}

}  // extern "C"
