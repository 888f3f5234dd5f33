// Internal structures shared by the host driver and the HIP kernels.
#pragma once

#include <string>
#include <vector>

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ctm.h"

namespace ctm {

constexpr int MAXD = CTM_MAXD;

// Operator classes of the stencil kernels.
//  HEAT: constant coefficients per axis (CTM_OP_HEAT).
//  SEP:  coefficients that depend on the coordinate of their own axis only,
//        read from 1-D tables (CTM_OP_OU, CTM_OP_CME).
//  VAR:  conservative variable-coefficient diffusion with
//        a = 1 + amp prod_k sin(2 pi x_k) at face midpoints (CTM_OP_VARCOEF).
//  DRIFT: Fokker-Planck operator with a full drift matrix: face velocities
//        depend on every coordinate; theta and H are read from the table
//        (CTM_OP_DRIFT).
enum OpClass { OPC_HEAT = 0, OPC_SEP = 1, OPC_VAR = 2, OPC_DRIFT = 3 };
enum SolverKind { SOLV_CG = 0, SOLV_BICG = 1 };

// Geometry of one component grid (device copy, read once per work-group).
struct GridDev {
  int npts;            // unknowns
  int d;
  int tabsz;           // doubles in this grid's coefficient table block
  int pad_;
  long long off;       // offset of the grid in a packed vector
  long long tab0;      // start of this grid's table block in the table arrays
  int n[MAXD];         // unknowns per axis (axis d-1 fastest)
  int stride[MAXD];    // point-index stride of axis i
  int tab[MAXD];       // offset of axis i inside the grid's table block
  int lev[MAXD];       // level l_i
  double ih2[MAXD];    // 1 / h_i^2
  double lo[MAXD];     // box lower corner
  double h[MAXD];      // mesh width
  int j0;              // node index of the first unknown (1 Dirichlet, 0 lattice)
  int pad3_;
  double coef;         // combination coefficient (-1)^w binom(d-1, w)
  // line layout of the on-chip solver: the stiffest axis `sax` is made the
  // fastest; internal point p = line * ns + j_sax, lines enumerate the other
  // axes oax[0..d-2] with oax[d-2] fastest
  int sax;             // stiff axis (canonical index)
  int ns;              // unknowns along the stiff axis
  int nlines;          // npts / ns
  int nseg;            // streaming solvers: segments per line of the line preconditioner
                       // (lines longer than kSegLen unknowns are cut into segments of
                       // kSegLen, the last one shorter; 1 otherwise)
  int oax[MAXD];       // non-stiff axes, canonical indices, increasing
  int lstride[MAXD];   // line-index stride of oax[m]
  int cstride[MAXD];   // canonical point stride of canonical axis i (= stride[i])
};

// Longest line segment the streaming solvers' line preconditioner solves
// exactly: 64 lanes of kSK = 16 unknowns (one wave). Longer lines are cut
// into segments of this length, solved exactly each, with the couplings
// between segments dropped from the preconditioner (block Jacobi over the
// segments; the operator keeps them).
constexpr int kSegLen = 1024;

// A family of packed vectors indexed by time: vector index = a * q + b
// (+ j for per-step roles); element (idx, grid g, point p) lives at
// base[idx * slen + g.off + p]. base == nullptr disables the role.
struct VecRef {
  double* base;
  long long a, b;
};

// Two-level overlapping Schwarz preconditioner (Section 2.1.2) of one grid:
// its subdomain records and index arrays (offsets into SchwarzView::ints),
// and its coarse inverse (offset into a level's coarse buffer).
struct SchwarzGrid {
  long long sub0;  // first subdomain record of the grid
  long long cord;  // curve order: grid point at each curve position (npts ints)
  long long cblk;  // coarse block of every grid point (npts ints)
  long long bst;   // first curve position of each coarse block (nblk + 1 ints)
  long long cinv;  // A_0^-1, nblk x nblk column-major (doubles)
  int nsub;        // subdomains P
  int nblk;        // coarse blocks
  int nmax;        // largest extended subdomain
  int pad_;
};
struct SchwarzSub {
  long long idx;   // grid points of the extended subdomain, curve order (n ints)
  long long srt;   // (point, local row) pairs sorted by point (2 n ints)
  long long inv;   // (R_i A R_i^T)^-1, n x n column-major (doubles, in a level's buffer)
  int n;           // unknowns of the extended subdomain
  int pad_;
  double omega;    // weight D_i = omega_i I
};
// What a launch needs of the preconditioner; grid == nullptr: the line
// preconditioner instead.
struct SchwarzView {
  const SchwarzGrid* grid;  // [G]
  const SchwarzSub* sub;
  const int* ints;
  const double* linv;       // local inverses of the launch's MGRIT level
  const double* cinv;       // coarse inverses of the launch's MGRIT level
  int balanced;             // 1: G^T C1 G + F (CG); 0: C1 + F (BiCGStab)
  int nbmax;                // largest coarse block count (LDS of a launch)
};
constexpr int kSchwarzMaxBlocks = 1024;
constexpr int kSchwarzMinS = 2, kSchwarzMaxS = 6;

// Arguments of one launch of the chain kernel. A task (g, q) takes grid g,
// loads the start vector of index start.a*q + start.b, applies `nsteps`
// implicit steps v <- Phi(v) + forcing_j and stores according to the roles.
struct ChainArgs {
  const GridDev* grids;
  const int2* tasks;        // (grid, q)
  const double* tab64;      // coefficient tables (FP64; FP32 copies are made in LDS)
  double amp;               // VAR amplitude
  double dt;                // step size of this level
  long long slen;           // length of a packed vector
  int nsteps;
  int maxit;                // Krylov iterations per solve / per refinement sweep
  int refine_maxit;
  int single32;             // mixed path: each step is one FP32 solve to inner_tol (no
                            // FP64 refinement); for loose coarse-level tolerances
  int fkind;                // forcing: 0 none, 1 manufactured heat problem (heat only)
  int resmode;              // MGRIT residual mode (both precisions): fixed-count steps,
                            // forcing before the step, exact space-time residual against a
                            // target
  double ft0, ftq;          // time of step j of task q: ft0 + q ftq + j dt
  double tol;               // FP64 path Krylov tolerance, or mixed refinement tolerance
  double inner_tol;         // mixed path FP32 Krylov tolerance
  VecRef start;             // start vector (base == nullptr: zero)
  VecRef start_wb;          // optional write-back of the start vector
  VecRef forcing;           // optional addend after step j: index a*q + b + j
  VecRef inter;             // optional store after step j < nsteps: index a*q + b + j
  VecRef fin;               // final store (index a*q + b)
  VecRef target;            // optional: residual mode, fin = v - target[a*q + b]
  VecRef guess;             // optional initial guess of step j < nsteps: index a*q + b + j
  VecRef guess_fin;         // optional initial guess of step nsteps: index a*q + b
  double* res2;             // residual mode: per-task ||fin||_2^2 (optional)
  unsigned long long* counters;  // statistics (see CNT_*)
  int* status;              // OR of (1 << ctm_status)
  const double* skip;       // optional: the launch does nothing once *skip != 0 (MGRIT
                            // work queued past the converged iteration)
  int pcrmax;               // cyclic-reduction steps the LDS of the launch holds per lane
                            // (at least log2 of the lanes per line of every grid of it)
  SchwarzView sch;          // streaming launches: the Schwarz preconditioner, if chosen
};

enum {
  CNT_KRYLOV = 0,
  CNT_KRYLOV_MAX = 1,
  CNT_REFINE = 2,
  CNT_REFINE_MAX = 3,
  CNT_SOLVES = 4,
  CNT_WORK = 5,
  CNT_DOFSTEPS = 6,  // implicit steps x unknowns
  CNT_N = 8
};

// Launch configurations of the on-chip solver: W waves per work-group, K
// consecutive stiff-axis unknowns per lane. A line of ns unknowns takes
// Lc = pow2ceil(ceil(ns / K)) <= 64 lanes of one wave.
struct ShapeCfg {
  int W, K;
};
constexpr ShapeCfg kShapes[] = {{1, 4}, {2, 4}, {4, 4}, {8, 4}, {16, 4},
                                {1, 8}, {2, 8}, {4, 8}, {8, 8}, {16, 8}};
constexpr int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);
// Grids beyond the on-chip shapes go to the streaming kernel (vectors in HBM
// scratch, one 1,024-thread work-group per task); its size class index:
constexpr int kStreamShape = kNumShapes;
// Statistics slot of the wide streaming solver (after the size classes).
constexpr int kWideSlot = kNumShapes + 1;
// Statistics slot of the on-chip launches that run in FP64 inside a mixed
// plan (its coarse MGRIT levels, all size classes together).
constexpr int kCoarse64Slot = kNumShapes + 2;
constexpr int kStatSlots = kNumShapes + 3;
static_assert(kStatSlots <= 16, "ctm_stats keeps 16 shape slots");

hipError_t launch_chain(int opc, int solver, bool mixed, int shape, const ChainArgs& a,
                        int ntasks, size_t smem, int tabmax, hipStream_t s);
// Streaming kernel (stream_ops.hip): task t of the launch uses the scratch
// doubles [t * SV_N * ss, (t + 1) * SV_N * ss); FP64 whatever the precision;
// d is the grids' dimension (selects the compile-time dimension bound).
constexpr int kStreamVectors = 14;
hipError_t launch_stream(int opc, int solver, int d, const ChainArgs& a, int ntasks, int tabmax,
                         double* scratch, long long ss, hipStream_t s);
hipError_t launch_stream_apply(int opc, int d, const GridDev* grids, int G, const double* tab64,
                               double amp, double dt, int tabmax, const double* x, double* y,
                               hipStream_t s);

// Wide streaming solver (wide_kernel.hpp, wide_ops.hip): the implicit steps
// of a few streaming tasks, each spread over many work-groups; one launch
// per Krylov phase, driven step by step from the host.
constexpr int kWT = 256;           // threads per point-wise work-group
constexpr int kWW = kWT / 64;      // its waves
constexpr int kWPT = 2;            // points per thread in the point-wise kernels
constexpr int kWP = kWT * kWPT;    // points per point-wise work-group
constexpr int kWLW = 1;            // waves per line work-group
constexpr int kWideSK = 16;        // unknowns per lane along a line (as the streaming kernel)
// static LDS of a line kernel of the wide solver (line tiles and sums); the
// coefficient tables (dynamic LDS) must fit beside it in 64 KiB
constexpr int kWideStaticLds = 20 * 1024;

// Sums of a task; each has a partial per producing work-group.
enum {
  WS_RR0 = 0,  // (r0, r0) of the step
  WS_BB,       // (b, b) of the step
  WS_RHV,      // (r^, v)
  WS_D = 3,    // t-phase of BiCGStab: WS_D + 5 parity + {ts, tt, ss, rhs, rht}
  WS_RR = 13,  // (r, r) after the update
  WS_PQ,       // CG: (p, q)
  WS_RZ = 15,  // CG: (r, z), WS_RZ + parity
  WS_FIN = 17, // ||fin||^2
  WS_N = 18
};

// Per-task state (device memory, one per task of the range).
struct WideTask {
  GridDev g;      // the task's grid (copied by the chain's first kernel)
  int q;          // the task's interval
  int fsrc;       // the task of the launch whose scratch holds this grid's line factors
  int done;       // the step's Krylov solve has stopped
  int it;         // its iteration count
  int pend;       // BiCGStab: breakdown found in the direction update
  int flag;       // status bits of the chain
  long long kr_sum, kr_max;
  double res_max;  // residual mode: max initial residual over the steps
};

struct WideArgs {
  ChainArgs a;
  double* scratch;  // task t of the range: scratch + t * SV_N * ss (as the streaming kernel)
  long long ss;
  WideTask* st;     // [tasks of the range]
  double* part;     // partial sums: [task][WS_N][maxblk]
  int maxblk;
  int j;            // step (1-based)
  int i;            // Krylov iteration
  int prev_its;     // iterations launched for the step being accounted
  int stage;        // line kernels stage contiguous lines through LDS
  int* host_out;    // poll: per task 1 while still iterating (mapped host memory)
};

// Kernels of the wide solver: SETUP (line factors, once per chain), STEP
// (step transition), INIT (initial residual), BA..BD (BiCGStab phases), CA..CC
// (CG phases), FIN (final store), FINISH (accounting, one wave per task),
// POLL (one wave per task: the next stopping test, busy flag to the host).
// SETUP, BA, BC and CA are line kernels.
enum WideKind { WK_SETUP = 0, WK_STEP, WK_INIT, WK_BA, WK_BB, WK_BC, WK_BD, WK_CA, WK_CB,
                WK_CC, WK_FIN, WK_FINISH, WK_POLL };
// grid: (work-groups per task, tasks).
hipError_t launch_wide(int opc, int solver, int d, int kind, const WideArgs& w, dim3 grid,
                       int tabmax, hipStream_t s);

// LDS copy of a vector the stencil reads: K rows (one per chunk position k)
// of pitch 64 W + kLdsGhost; thread t owns column t, and the columns from
// 64 W on hold zeros that lanes without a neighbour line read instead.
constexpr int kLdsGhost = 2;
__host__ __device__ constexpr int lds_pitch(int W) { return 64 * W + kLdsGhost; }

// Constant-coefficient operator (OPC_HEAT), one table per work-group and
// precision in LDS: the stencil weights, and the line preconditioner's
// factors, which are the same for every line of the grid: the elimination
// factors of a chunk's interior (shared by all chunks; a chunk scales the
// responses phiU/psiU by its own couplings) and the cyclic-reduction factors
// of each lane position c of a line.
constexpr int kMaxPcr = 6;  // log2(64): cyclic-reduction steps over <= 64 lanes
template <typename T, int K>
struct HeatTab {
  T diag, s;            // diagonal of A, coupling along the stiff axis
  T o[MAXD - 1];        // coupling to the neighbour lines along oax[m]
  T m[K], id[K], cu[K]; // Thomas multipliers, reciprocal pivots, upper couplings
  T phiU[K], psiU[K];   // interior responses to the previous / own interface unknown
  T pa[kMaxPcr][64], pc[kMaxPcr][64], pinv[64];  // per lane position c
};

// Dynamic LDS of the chain kernel: FP64 vector, FP32 vector (mixed), the
// coefficient tables (FP64, then FP32 if mixed), the constant-coefficient
// tables (heat; FP64, then FP32 if mixed), the uniform off-axis couplings
// of the variable-coefficient operator (FP64 and FP32), two reduction slots,
// and the cyclic-reduction factors of the line preconditioner (operators with
// per-line coefficients, in the precision the preconditioner runs in):
// row 0 the reciprocal reduced diagonal, rows 1 + 2r and 2 + 2r the factors
// of step r, one column per thread.
struct ChainSmem {
  size_t x32, tab, heat, ocv, red, pre, op, total;  // byte offsets and total
};
// Doubles per lane of the FP64 variable-coefficient line operator that a
// mixed chain keeps in LDS: its faces (K + 1) and off-axis factors (qlo,
// qup: MAXD - 1 each); the diagonal and the node sines stay in registers.
// (Parking those as well measured no faster, even in eight-wave work-groups
// whose LDS has room for them.)
__host__ __device__ constexpr int parked_op_words(int K) { return K + 1 + 2 * (MAXD - 1); }
__host__ __device__ constexpr size_t align16(size_t b) { return (b + 15) & ~size_t(15); }
__host__ __device__ constexpr size_t heat_tab_bytes(int K, bool mixed) {
  return K == 4 ? align16(sizeof(HeatTab<double, 4>)) +
                      (mixed ? align16(sizeof(HeatTab<float, 4>)) : 0)
                : align16(sizeof(HeatTab<double, 8>)) +
                      (mixed ? align16(sizeof(HeatTab<float, 8>)) : 0);
}
constexpr size_t kOcvBytes = MAXD * sizeof(double) + MAXD * sizeof(float);
// rows of the cyclic-reduction table for pcr steps (0: no table)
__host__ __device__ constexpr int pcr_rows(int pcr) { return pcr < 0 ? 0 : 2 * pcr + 1; }
// park: the FP64 line operator of a mixed variable-coefficient chain lives in
// LDS (see the chain kernel), after the cyclic-reduction table.
__host__ __device__ constexpr ChainSmem chain_smem_layout(int W, int K, int tabmax, bool mixed,
                                                          bool heat, int pcr, bool park = false) {
  const size_t elems = (size_t)K * lds_pitch(W);
  const size_t x32 = align16(elems * sizeof(double));
  const size_t tab = x32 + (mixed ? align16(elems * sizeof(float)) : 0);
  const size_t hb = tab + align16((size_t)tabmax * sizeof(double) +
                                  (mixed ? (size_t)tabmax * sizeof(float) : 0));
  const size_t ocv = hb + (heat ? heat_tab_bytes(K, mixed) : 0);
  const size_t red = ocv + align16(kOcvBytes);
  const size_t pre = red + 2u * 64u * sizeof(double);
  const size_t prebytes =
      heat ? 0 : align16((size_t)pcr_rows(pcr) * 64u * W * (mixed ? sizeof(float) : sizeof(double)));
  const size_t op = pre + prebytes;
  const size_t opbytes = park ? align16((size_t)parked_op_words(K) * 64u * W * sizeof(double)) : 0;
  return ChainSmem{x32, tab, hb, ocv, red, pre, op, op + opbytes};
}
inline size_t chain_smem_bytes(int shape, int tabmax, bool mixed, bool heat, int pcr,
                               bool park = false) {
  return chain_smem_layout(kShapes[shape].W, kShapes[shape].K, tabmax, mixed, heat, pcr, park)
      .total;
}

// Auxiliary kernels (aux_kernels.hip).
hipError_t launch_initial_state(const GridDev* grids, int G, int maxpts, int nlev, int terms,
                                const double* icw, const double* icf, double* out, hipStream_t s);
// u*(x, t) of the manufactured heat problem at every unknown.
hipError_t launch_mms_initial(const GridDev* grids, int G, int maxpts, double t, double* out,
                              hipStream_t s);
hipError_t launch_apply(int opc, int shape, const GridDev* grids, int G, const double* tab64,
                        double amp, double dt, int tabmax, const double* x, double* y,
                        hipStream_t s);
// Combination gather. stages: runs of consecutive grids [x, y) whose
// unknowns fit gather_stage_capacity() doubles (a larger grid alone); d: the
// plan's dimension.
hipError_t launch_gather(const GridDev* grids, const int2* stages, int nstage, int d,
                         const double* u, const double* pts, long long npts, double* out,
                         hipStream_t s);
int gather_stage_capacity();
hipError_t launch_project(const GridDev* grids, const long long* offsets, int G, long long slen,
                          const double* u, double* out, hipStream_t s);
// Hierarchical basis (Section 2.2.2): per-grid (de)hierarchization (one
// work-group per grid, the grid staged in LDS; in may equal out), the
// combination of surpluses per basis function, sg[s] = sum over the entries
// e of node s of coef[e] * uh[idx[e]], and the scatter out[p] = sg[node[p]].
hipError_t launch_hierarchize(const GridDev* grids, int G, int maxpts, bool lattice,
                              bool inverse, const double* in, double* out, hipStream_t s);
hipError_t launch_hier_combine(const int* off, const int* idx, const double* coef, int nodes,
                               const double* uh, double* sg, hipStream_t s);
hipError_t launch_hier_scatter(const int* node, long long slen, const double* sg, double* out,
                               hipStream_t s);
hipError_t launch_grid_norms2(const GridDev* grids, int G, const double* u, double* out,
                              hipStream_t s);
// MGRIT convergence test of iteration it on the device: res = max over tasks
// t of sqrt(res2[t] / norm2[grid(t)]) (norm2 = 0 -> 1). Unless mg[0] (the
// stopping iteration, 0 while running) is set already, mg[2 it] = res and
// mg[0] = it when res <= tol, res is not a number, or *status has the
// non-finite bit. Always mg[2 it + 1] = mg[0]. host_mg (optional, mapped
// pinned host memory) receives mg[2 it] and mg[2 it + 1] as well.
hipError_t launch_residual_max(const int2* tasks, int ntasks, const double* res2,
                               const double* norm2, double* part, double* mg, double* host_mg,
                               int it, double tol, const int* status, hipStream_t s);
// partial maxima the residual test needs in the workspace (doubles)
constexpr int kResBlocks = 256;
// dst[(ad q + bd) slen + e] = x[(ax q + bx) slen + e] (+ y[(ay q + by) slen + e]),
// q = 0..nvec-1, e = 0..slen-1; y.base may be null.
// skip (optional): the launch does nothing once *skip != 0.
hipError_t launch_vec_add(VecRef dst, VecRef x, VecRef y, int nvec, long long slen,
                          hipStream_t s, const double* skip = nullptr);
// The same restricted to the unknowns of the grids tasks[0..ntasks).x (one
// size class): vectors q = 0..nvec-1, only the entries of those grids; x.base
// may be null as well (then dst = y, or zero).
hipError_t launch_class_vec_add(const int2* tasks, int ntasks, const GridDev* grids, VecRef dst,
                                VecRef x, VecRef y, int nvec, long long slen, hipStream_t s,
                                const double* skip);
hipError_t launch_fill_zero(double* p, long long n, hipStream_t s,
                            const double* skip = nullptr);

// ------------------------------------------------ Schwarz preconditioner
// Host decomposition of one grid (Section 2.1.2): Hilbert-curve order of
// the unknowns with virtual nodes, disjoint partition, overlap, weights and
// coarse blocks. Appends the grid's subdomain records and index arrays to
// `subs` / `ints` and fills `sg` (offsets into those; `sg.cinv` and the
// records' `inv` are offsets into the per-level inverse buffers, advanced in
// `linv_len` / `cinv_len`). Returns false (and a message) when the grid
// exceeds the preconditioner's limits.
bool schwarz_decompose(const GridDev& gd, int S, SchwarzGrid& sg, std::vector<SchwarzSub>& subs,
                       std::vector<int>& ints, long long& linv_len, long long& cinv_len,
                       std::string& msg);
// Device set-up of one MGRIT level (step dt): the dense local matrices
// R_i A R_i^T of every subdomain (records subs[0..nsub_total), owner grid
// sub_grid[i]) into linv, the coarse matrices R_0 A R_0^T of every grid into
// cinv, then both inverted in place (Gauss-Jordan with partial pivoting);
// *status gets the breakdown bit for a singular pivot.
hipError_t launch_schwarz_setup(int opc, int d, const GridDev* grids, int G, const double* tab64,
                                double amp, double dt, int tabmax, const SchwarzView& v,
                                double* linv, double* cinv, const int* sub_grid,
                                long long nsub_total, int nmax_sub, int* status,
                                hipStream_t s);
// y = C x on every grid (one work-group per grid) with the Schwarz
// preconditioner of the view's level; scratch holds kStreamVectors vectors
// of ss doubles per grid.
hipError_t launch_schwarz_apply(int opc, int solver, int d, const GridDev* grids, int G,
                                const double* tab64, double amp, double dt, int tabmax,
                                const SchwarzView& v, const double* x, double* y,
                                double* scratch, long long ss, hipStream_t s);

}  // namespace ctm
