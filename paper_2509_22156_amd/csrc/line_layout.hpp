// Line layout of the on-chip solver and its line-block preconditioner.
//
// Each grid is traversed along its stiffest axis s (largest coupling, i.e.
// finest mesh width): a "line" is the set of ns unknowns with fixed
// coordinates on the other axes. A line is split into chunks of K
// consecutive unknowns; chunk c of a line lives in lane c of a segment of
// Lc = pow2ceil(ceil(ns / K)) consecutive lanes of one wave, so neighbours
// along s are in the lane's own registers or in the adjacent lane
// (cross-lane shuffle), and only the other axes go through LDS.
//
// Preconditioner: M = the part of A = I + dt L that couples unknowns along
// s (block Jacobi with whole lines as blocks, i.e. a non-overlapping
// decomposition into line subdomains with exact subdomain solves; the
// paper's own spatial solver is a Krylov method preconditioned by domain
// decomposition with exact local solves, Section 2.1.2). M^-1 is applied
// exactly: Thomas elimination of each chunk's first K-1 unknowns in
// registers, a tridiagonal interface system with one unknown per lane (the
// chunk's last unknown) solved by parallel cyclic reduction over the
// lanes of the line, and back-substitution. All matrix-only factors are
// computed once per chain (per step size).
#pragma once

#include <type_traits>

#include "device_common.hpp"

namespace ctm {

// ------------------------------------------------------------- shuffles
// Lane exchanges inside a line segment of Lc lanes (Lc a power of two,
// segments aligned). Shifts by one lane use the wave-wide DPP shifts; shifts
// by 2..8 inside segments of at most 16 lanes stay within a DPP row; longer
// shifts go through ds_bpermute. Lanes whose source lies outside their
// segment receive an unspecified value and must be masked by the caller.
template <typename T>
__device__ __forceinline__ T from_minus(T v, int s, int Lc) {
  if (s == 1) return dpp<0x138>(v);  // wave_shr:1
  if (Lc <= 16) {
    switch (s) {
      case 2: return dpp<0x112>(v);  // row_shr:2
      case 4: return dpp<0x114>(v);
      case 8: return dpp<0x118>(v);
      default: break;
    }
  }
  return __shfl_up(v, (unsigned)s, Lc);
}
template <typename T>
__device__ __forceinline__ T from_plus(T v, int s, int Lc) {
  if (s == 1) return dpp<0x130>(v);  // wave_shl:1
  if (Lc <= 16) {
    switch (s) {
      case 2: return dpp<0x102>(v);  // row_shl:2
      case 4: return dpp<0x104>(v);
      case 8: return dpp<0x108>(v);
      default: break;
    }
  }
  return __shfl_down(v, (unsigned)s, Lc);
}

__device__ __forceinline__ int pow2ceil(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

// Position of this lane in the line layout of grid g.
template <int K>
struct Lane {
  int line;        // line index (>= nlines: idle lane)
  int c;           // chunk index inside the line
  int Lc;          // lanes per line
  int j0;          // stiff coordinate of the chunk's first unknown (c * K)
  int nval;        // unknowns of the chunk inside the line (0..K)
  int tid;         // thread index: LDS slot of unknown k is k * lds_pitch(W) + tid
  long long cbase; // canonical index of the chunk's first unknown
  int cstep;       // canonical stride along the stiff axis
  bool nxt;        // the next chunk of the line holds unknowns
  unsigned nb;     // bit 2m: lower neighbour line along oax[m]; bit 2m+1: upper
  int jo[MAXD];    // coordinates on the non-stiff axes oax[m]
};

template <int K>
__device__ __forceinline__ void setup_lane(const GridDev& g, Lane<K>& L) {
  const int Lc = pow2ceil((g.ns + K - 1) / K);
  const int t = threadIdx.x;
  const int lane = t & 63;
  L.Lc = Lc;
  L.c = lane & (Lc - 1);
  L.line = (t >> 6) * (64 / Lc) + lane / Lc;
  L.j0 = L.c * K;
  const bool live = L.line < g.nlines;
  int nv = g.ns - L.j0;
  nv = nv < 0 ? 0 : (nv > K ? K : nv);
  L.nval = live ? nv : 0;
  L.tid = t;
  L.nxt = live && (L.j0 + K < g.ns);
  L.cstep = g.cstride[g.sax];
  long long cb = 0;
  unsigned nb = 0;
  int rem = live ? L.line : 0;
#pragma unroll
  for (int m = 0; m < MAXD - 1; ++m) {
    L.jo[m] = 0;
    if (m < g.d - 1) {
      const int ax = g.oax[m];
      const int j = (rem / g.lstride[m]) % g.n[ax];
      L.jo[m] = j;
      cb += (long long)j * g.cstride[ax];
      nb |= (unsigned)(j > 0) << (2 * m);
      nb |= (unsigned)(j < g.n[ax] - 1) << (2 * m + 1);
    }
  }
  L.cbase = cb + (long long)L.j0 * L.cstep;
  L.nb = live ? nb : 0u;
}

// ---------------------------------------------------------- operators
// Coefficients of A = I + dt L in the line layout, precision T:
//  diag[k]        diagonal of the chunk's unknown k
//  slo[k], sup[k] couplings to the stiff-axis neighbours j-1, j+1
//  olo[m], oup[m] couplings to the neighbour lines along oax[m] (per lane;
//                 VAR adds a per-unknown part qlo/qup[m] * snj[k])
template <int OPC, typename T, int K>
struct LineOp {
  T diag[K];
  T slo[K];
  T sup[K];
  T olo[MAXD - 1], oup[MAXD - 1];
  T qlo[OPC == OPC_VAR ? MAXD - 1 : 1], qup[OPC == OPC_VAR ? MAXD - 1 : 1];
  T snj[OPC == OPC_VAR ? K : 1];
};
// HEAT: the weights are the same for every lane; they live in the
// work-group's LDS table (read with broadcast loads), not in registers.
template <typename T, int K>
struct LineOp<OPC_HEAT, T, K> {
  HeatTab<T, K>* h;
};
// VAR: the coupling along the stiff axis between unknowns k-1 and k is the
// face value face[k] (shared by both unknowns, the operator is symmetric);
// the coupling to the neighbour line along oax[m] at unknown k is
// oc[m] + q{lo,up}[m] * snj[k]: a part -dt/h_m^2 that is the same for the
// whole grid (a work-group table in LDS, oc) and a per-lane factor times the
// stiff-axis node sine of the unknown.
template <typename T, int K>
struct LineOp<OPC_VAR, T, K> {
  T diag[K];
  T face[K + 1];
  T snj[K];
  T qlo[MAXD - 1], qup[MAXD - 1];
  const T* oc;
};
// DRIFT: second-order central differences (conservative central face
// fluxes w (u_j + u_{j+1}) / 2, central diffusion). The face velocity along a
// non-stiff axis a at unknown k is
// base[m] + theta[a][s] x_s(k) -/+ theta[a][a] h_a / 2, so a lane keeps
// base[m] (the contribution of its fixed coordinates) and computes the
// neighbour couplings in the apply; the stiff-axis and diagonal couplings
// are kept per unknown.
template <typename T, int K>
struct LineOp<OPC_DRIFT, T, K> {
  T diag[K], slo[K], sup[K];
  T base[MAXD - 1];  // sum over the non-stiff axes c of theta[oax[m]][c] x_c
  T xs0;             // stiff coordinate of the chunk's first unknown
  T dt;
  const T* tab;      // theta (row-major d x d), then H (d), in LDS
};

// tab: this grid's tables in LDS (SEP: per axis Lo, D, Up of L scaled by
// dt; VAR: per axis node sines then face sines). ht: the work-group's
// constant-coefficient table (HEAT only; thread 0 fills its weights, and a
// barrier must follow before they are read). ocv: the work-group's table of
// uniform off-axis couplings (VAR only; thread 0 fills it, and a barrier
// must follow before the first apply reads it).
template <int OPC, typename T, int K>
__device__ __forceinline__ void lineop_setup(const GridDev& g, const Lane<K>& L, double dt,
                                             double amp, const T* tab, HeatTab<T, K>* ht,
                                             T* ocv, LineOp<OPC, T, K>& O) {
  const int s = g.sax;
  const double cs = dt * g.ih2[s];
  if constexpr (OPC == OPC_HEAT) {
    O.h = ht;
    if (threadIdx.x == 0) {
      double sum = 0.0;
#pragma unroll
      for (int i = 0; i < MAXD; ++i) sum += (i < g.d) ? 2.0 * dt * g.ih2[i] : 0.0;
      ht->diag = (T)(1.0 + sum);
      ht->s = (T)(-cs);
#pragma unroll
      for (int m = 0; m < MAXD - 1; ++m)
        ht->o[m] = (T)(-((m < g.d - 1) ? dt * g.ih2[g.oax[m]] : 0.0));
    }
  } else if constexpr (OPC == OPC_DRIFT) {
    const int d = g.d;
    O.tab = tab;
    O.dt = (T)dt;
    T xo[MAXD - 1];
#pragma unroll
    for (int m = 0; m < MAXD - 1; ++m)
      xo[m] = (m < d - 1) ? (T)(g.lo[g.oax[m]] + (double)(L.jo[m] + g.j0) * g.h[g.oax[m]])
                          : (T)0;
    T bs = (T)0;  // stiff-axis velocity without the stiff coordinate
#pragma unroll
    for (int m = 0; m < MAXD - 1; ++m) {
      O.base[m] = (T)0;
      if (m < d - 1) {
        const int a = g.oax[m];
        T acc = (T)0;
#pragma unroll
        for (int mm = 0; mm < MAXD - 1; ++mm)
          if (mm < d - 1) acc += tab[a * d + g.oax[mm]] * xo[mm];
        O.base[m] = acc;
        bs += tab[s * d + a] * xo[m];
      }
    }
    const T hs = (T)g.h[s];
    O.xs0 = (T)(g.lo[s] + (double)(L.j0 + g.j0) * g.h[s]);
    const T tss = tab[s * d + s], Hs = tab[d * d + s];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const bool v = k < L.nval;
      const T xs = O.xs0 + (T)k * hs;
      const T wc = bs + tss * xs;
      const T wup = wc + tss * (T)0.5 * hs, wdn = wc - tss * (T)0.5 * hs;
      T dg = (T)0.5 * (wup - wdn) / hs + Hs / (hs * hs);
      const T up = (T)0.5 * wup / hs - (T)0.5 * Hs / (hs * hs);
      const T lo = (T)-0.5 * wdn / hs - (T)0.5 * Hs / (hs * hs);
#pragma unroll
      for (int m = 0; m < MAXD - 1; ++m) {
        if (m < d - 1) {
          const int a = g.oax[m];
          const T ha = (T)g.h[a], taa = tab[a * d + a];
          const T w0 = O.base[m] + tab[a * d + s] * xs;
          const T wu = w0 + taa * (T)0.5 * ha, wd = w0 - taa * (T)0.5 * ha;
          dg += (T)0.5 * (wu - wd) / ha + tab[d * d + a] / (ha * ha);
        }
      }
      O.diag[k] = v ? (T)1 + O.dt * dg : (T)1;
      O.slo[k] = v ? O.dt * lo : (T)0;
      O.sup[k] = v ? O.dt * up : (T)0;
    }
  } else if constexpr (OPC == OPC_SEP) {
    T dl = (T)1;
#pragma unroll
    for (int m = 0; m < MAXD - 1; ++m) {
      O.olo[m] = (T)0;
      O.oup[m] = (T)0;
      if (m < g.d - 1) {
        const int ax = g.oax[m];
        const T* t = tab + g.tab[ax];
        const int j = L.jo[m];
        O.olo[m] = t[j];
        dl += t[g.n[ax] + j];
        O.oup[m] = t[2 * g.n[ax] + j];
      }
    }
    const T* t = tab + g.tab[s];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int j = L.j0 + k;
      const bool v = k < L.nval;
      O.diag[k] = v ? dl + t[g.n[s] + j] : (T)1;
      O.slo[k] = v ? t[j] : (T)0;
      O.sup[k] = v ? t[2 * g.n[s] + j] : (T)0;
    }
  } else {
    // a = 1 + amp * (face sine) * (product of node sines of the other axes)
    T sn[MAXD - 1];
#pragma unroll
    for (int m = 0; m < MAXD - 1; ++m)
      sn[m] = (m < g.d - 1) ? tab[g.tab[g.oax[m]] + L.jo[m]] : (T)1;
    T pre[MAXD - 1], suf[MAXD - 1];
    T run = (T)1;
#pragma unroll
    for (int m = 0; m < MAXD - 1; ++m) {
      pre[m] = run;
      run *= sn[m];
    }
    const T es = run;  // product over all non-stiff axes
    run = (T)1;
#pragma unroll
    for (int m = MAXD - 2; m >= 0; --m) {
      suf[m] = run;
      run *= sn[m];
    }
    const T A = (T)amp;
    O.oc = ocv;
    if (threadIdx.x == 0) {
#pragma unroll
      for (int m = 0; m < MAXD - 1; ++m)
        ocv[m] = (m < g.d - 1) ? (T)(-(dt * g.ih2[g.oax[m]])) : (T)0;
    }
    T diag_lane = (T)1;  // 1 + sum_m (dt/h_m^2) (a_lo + a_up) without the snj parts
    T qsum = (T)0;       // sum_m (qlo[m] + qup[m]): the snj-proportional diagonal part
#pragma unroll
    for (int m = 0; m < MAXD - 1; ++m) {
      O.qlo[m] = (T)0;
      O.qup[m] = (T)0;
      if (m < g.d - 1) {
        const int ax = g.oax[m];
        const T cm = (T)(dt * g.ih2[ax]);
        const T* sm = tab + g.tab[ax] + g.n[ax];
        const T pm = pre[m] * suf[m];
        O.qlo[m] = -cm * A * sm[L.jo[m]] * pm;
        O.qup[m] = -cm * A * sm[L.jo[m] + 1] * pm;
        diag_lane += cm + cm;
        qsum += O.qlo[m] + O.qup[m];
      }
    }
    const T* sns = tab + g.tab[s];
    const T* sms = tab + g.tab[s] + g.n[s];
    const T csT = (T)cs;
    // faces j0 .. j0 + nval of the chunk (face k lies below unknown k)
#pragma unroll
    for (int k = 0; k <= K; ++k)
      O.face[k] = (L.nval > 0 && k <= L.nval) ? -csT * ((T)1 + A * sms[L.j0 + k] * es) : (T)0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const bool v = k < L.nval;
      const T snv = v ? sns[L.j0 + k] : (T)0;
      O.snj[k] = snv;
      O.diag[k] = v ? diag_lane - (O.face[k] + O.face[k + 1]) - qsum * snv : (T)1;
    }
  }
}

// The FP64 variable-coefficient line operator of a mixed chain, partly
// parked in LDS: the faces and the off-axis factors (parked_op_words(K) per
// lane) go to LDS, field-major with lane-consecutive slots (word e of
// thread t at lds[e * BS + t]: every wave access is conflict-free); the
// diagonal and the node sines stay in registers (LineOpVarKeep). The chain
// keeps it that way through the FP32 inner solves and loads the parked part
// back for each FP64 residual.
template <int K>
struct LineOpVarKeep {
  double diag[K];
  double snj[K];
};
template <int K, int BS>
__device__ __forceinline__ void lineop_park(const LineOp<OPC_VAR, double, K>& O, double* lds,
                                            LineOpVarKeep<K>& keep) {
  const int t = threadIdx.x;
  int e = 0;
#pragma unroll
  for (int k = 0; k <= K; ++k) lds[(e++) * BS + t] = O.face[k];
#pragma unroll
  for (int m = 0; m < MAXD - 1; ++m) lds[(e++) * BS + t] = O.qlo[m];
#pragma unroll
  for (int m = 0; m < MAXD - 1; ++m) lds[(e++) * BS + t] = O.qup[m];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    keep.diag[k] = O.diag[k];
    keep.snj[k] = O.snj[k];
  }
}
template <int K, int BS>
__device__ __forceinline__ void lineop_unpark(LineOp<OPC_VAR, double, K>& O, const double* lds,
                                              const LineOpVarKeep<K>& keep, const double* oc) {
  const int t = threadIdx.x;
  int e = 0;
#pragma unroll
  for (int k = 0; k <= K; ++k) O.face[k] = lds[(e++) * BS + t];
#pragma unroll
  for (int m = 0; m < MAXD - 1; ++m) O.qlo[m] = lds[(e++) * BS + t];
#pragma unroll
  for (int m = 0; m < MAXD - 1; ++m) O.qup[m] = lds[(e++) * BS + t];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    O.diag[k] = keep.diag[k];
    O.snj[k] = keep.snj[k];
  }
  O.oc = oc;
}

template <int OPC, typename T, int K>
__device__ __forceinline__ T op_diag(const LineOp<OPC, T, K>& O, int k) {
  if constexpr (OPC == OPC_HEAT) return O.h->diag;
  else return O.diag[k];
}
template <int OPC, typename T, int K>
__device__ __forceinline__ T op_slo(const LineOp<OPC, T, K>& O, int k) {
  if constexpr (OPC == OPC_HEAT) return O.h->s;
  else if constexpr (OPC == OPC_VAR) return O.face[k];
  else return O.slo[k];
}
template <int OPC, typename T, int K>
__device__ __forceinline__ T op_sup(const LineOp<OPC, T, K>& O, int k) {
  if constexpr (OPC == OPC_HEAT) return O.h->s;
  else if constexpr (OPC == OPC_VAR) return O.face[k + 1];
  else return O.sup[k];
}
template <int OPC, typename T, int K>
__device__ __forceinline__ T op_olo(const LineOp<OPC, T, K>& O, int m) {
  if constexpr (OPC == OPC_HEAT) return O.h->o[m];
  else if constexpr (OPC == OPC_VAR) return O.oc[m];
  else return O.olo[m];
}
template <int OPC, typename T, int K>
__device__ __forceinline__ T op_oup(const LineOp<OPC, T, K>& O, int m) {
  if constexpr (OPC == OPC_HEAT) return O.h->o[m];
  else if constexpr (OPC == OPC_VAR) return O.oc[m];
  else return O.oup[m];
}

// Write the chunk to LDS, transposed: unknown k of thread t goes to slot
// k * pitch + t, so that every LDS access of a wave touches consecutive
// addresses (no bank conflicts). A barrier must follow before line_apply.
// Thread t holds chunk c of line `line` with t = line * Lc + c, so the
// neighbouring line along oax[m] lives in thread t +- lstride[m] * Lc.
template <typename T, int K, int PITCH>
__device__ __forceinline__ void lds_put(const Lane<K>& L, T* xl, const T (&x)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) xl[k * PITCH + L.tid] = x[k];
}

// Zero the ghost columns (column blockDim.x + i of every row); done once per
// kernel before the first barrier, never overwritten by lds_put.
template <typename T, int K>
__device__ __forceinline__ void lds_zero_ghosts(T* xl) {
  const int t = threadIdx.x;
  if (t < K * kLdsGhost)
    xl[(t / kLdsGhost) * ((int)blockDim.x + kLdsGhost) + (int)blockDim.x + t % kLdsGhost] = (T)0;
}

// y = A x on the chunk; xl holds x of the whole grid (after a barrier).
// Padding entries of x (k >= nval) must be zero, and so are those of y. A
// missing neighbour line is read from the zero ghost column.
template <int OPC, typename T, int K, int PITCH>
__device__ __forceinline__ void line_apply(const GridDev& g, const Lane<K>& L,
                                           const LineOp<OPC, T, K>& O, const T* xl,
                                           const T (&x)[K], T (&y)[K]) {
  const T xleft = from_minus(x[K - 1], 1, L.Lc);
  const T xright = from_plus(x[0], 1, L.Lc);
  T acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const T xm = (k > 0) ? x[k - 1] : (L.c > 0 ? xleft : (T)0);
    const T xp = (k < K - 1) ? x[k + 1] : (L.nxt ? xright : (T)0);
    acc[k] = op_diag(O, k) * x[k] + op_slo(O, k) * xm + op_sup(O, k) * xp;
  }
  // PITCH (the LDS row length) is a compile-time constant, so the K row
  // offsets of a neighbour read are immediate fields of the LDS loads
  const int ghost = PITCH - kLdsGhost;
#pragma unroll
  for (int m = 0; m < MAXD - 1; ++m) {
    if (m < g.d - 1) {
      const int off = g.lstride[m] * L.Lc;
      const T* plo = xl + (((L.nb >> (2 * m)) & 1u) ? L.tid - off : ghost);
      const T* phi = xl + (((L.nb >> (2 * m + 1)) & 1u) ? L.tid + off : ghost);
      if constexpr (OPC == OPC_DRIFT) {
        // central-flux couplings from the face velocities of this unknown
        const int d = g.d, a = g.oax[m], s = g.sax;
        const T ha = (T)g.h[a], hs = (T)g.h[s];
        const T tas = O.tab[a * d + s], half = O.tab[a * d + a] * (T)0.5 * ha;
        const T ih = (T)0.5 * O.dt / ha;
        const T dH = (T)0.5 * O.dt * O.tab[d * d + a] / (ha * ha);
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const T w0 = O.base[m] + tas * (O.xs0 + (T)k * hs);
          const T clo = -ih * (w0 - half) - dH;
          const T chi = ih * (w0 + half) - dH;
          acc[k] += clo * plo[k * PITCH];
          acc[k] += chi * phi[k * PITCH];
        }
      } else {
#pragma unroll
        for (int k = 0; k < K; ++k) {
          T clo = op_olo(O, m), chi = op_oup(O, m);
          if constexpr (OPC == OPC_VAR) {
            clo += O.qlo[m] * O.snj[k];
            chi += O.qup[m] * O.snj[k];
          }
          acc[k] += clo * plo[k * PITCH];
          acc[k] += chi * phi[k * PITCH];
        }
      }
    }
  }
#pragma unroll
  for (int k = 0; k < K; ++k) y[k] = (k < L.nval) ? acc[k] : (T)0;
}

// ------------------------------------------------------ preconditioner
// Per-lane factors of the chunk interior in registers; the cyclic-reduction
// factors of the interface system live in a work-group table in LDS (one
// column per thread, row stride BS: row 0 the reciprocal reduced diagonal,
// rows 1 + 2r and 2 + 2r the factors of step r), read back by the same
// thread only, so no barrier is needed between setup and use.
// The Thomas multipliers m_k = a_k / pivot_{k-1} and the upper couplings c_k
// of the chunk interior are the operator's own couplings times the stored
// reciprocal pivots, so they are formed from the LineOp in the apply rather
// than kept in registers.
template <typename T, int K>
struct LinePre {
  T id[K];           // reciprocal pivots (k = 0..K-2)
  T phi[K], psi[K];  // interior responses to the previous / own interface unknown
  T aL, cL;          // couplings of the chunk's last unknown
  T* pl;             // this thread's column of the cyclic-reduction table
  int steps;         // log2(Lc)
};

// pre: the work-group's cyclic-reduction table (pcrmax steps); a grid whose
// lines need more steps than the table holds raises FLAG_INVALID in *flag
// and is left unpreconditioned along its interface (the launch reports an
// error; the host sizes the table so that this does not happen).
template <int OPC, typename T, int K, int BS>
__device__ __forceinline__ void linepre_setup(const Lane<K>& L, const LineOp<OPC, T, K>& O,
                                              LinePre<T, K>& M, T* pre, int pcrmax,
                                              int* flag) {
  static_assert(K >= 2, "chunks hold at least two unknowns");
  T a[K], b[K], c[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const bool v = k < L.nval;
    const int j = L.j0 + k;
    a[k] = (v && j > 0) ? op_slo(O, k) : (T)0;
    c[k] = (v && k + 1 < L.nval) ? op_sup(O, k) : (T)0;
    b[k] = v ? op_diag(O, k) : (T)1;
  }
  T mm[K];
  mm[0] = (T)0;
  M.id[0] = (T)1 / b[0];
#pragma unroll
  for (int k = 1; k < K - 1; ++k) {
    mm[k] = a[k] * M.id[k - 1];
    M.id[k] = (T)1 / (b[k] - mm[k] * c[k - 1]);
  }
  // phi = T_I^-1 (a_0 e_0), psi = T_I^-1 (c_{K-2} e_{K-2})
  T f[K];
  f[0] = a[0];
#pragma unroll
  for (int k = 1; k < K - 1; ++k) f[k] = -mm[k] * f[k - 1];
  M.phi[K - 2] = f[K - 2] * M.id[K - 2];
#pragma unroll
  for (int k = K - 3; k >= 0; --k) M.phi[k] = (f[k] - c[k] * M.phi[k + 1]) * M.id[k];
  M.psi[K - 2] = c[K - 2] * M.id[K - 2];
#pragma unroll
  for (int k = K - 3; k >= 0; --k) M.psi[k] = -c[k] * M.psi[k + 1] * M.id[k];
  M.phi[K - 1] = (T)0;
  M.psi[K - 1] = (T)0;
  // interface equation of the chunk's last unknown u_c:
  //   A u_{c-1} + B u_c + C u_{c+1} = R
  // its coupling to the next chunk: the stiff-axis neighbour j0+K exists
  // iff this chunk is full and the next one holds unknowns
  const T phi0n = from_plus(M.phi[0], 1, L.Lc);
  const T psi0n = from_plus(M.psi[0], 1, L.Lc);
  const bool has_next = L.nxt;
  M.aL = (L.nval == K && K - 1 + L.j0 > 0) ? a[K - 1] : (T)0;
  M.cL = has_next ? op_sup(O, K - 1) : (T)0;
  T A = -M.aL * M.phi[K - 2];
  T B = b[K - 1] - M.aL * M.psi[K - 2] - M.cL * phi0n;
  T C = -M.cL * psi0n;
  M.pl = pre + threadIdx.x;
  // cyclic reduction factors over the Lc lanes of the line
  int steps = 0;
  while ((1 << steps) < L.Lc) ++steps;
  if (steps > pcrmax) {
    *flag |= FLAG_INVALID;
    steps = pcrmax;
  }
  M.steps = steps;
#pragma unroll
  for (int r = 0; r < kMaxPcr; ++r) {
    const int s = 1 << r;
    if (r < steps) {
      const T Am = from_minus(A, s, L.Lc), Bm = from_minus(B, s, L.Lc),
              Cm = from_minus(C, s, L.Lc);
      const T Ap = from_plus(A, s, L.Lc), Bp = from_plus(B, s, L.Lc),
              Cp = from_plus(C, s, L.Lc);
      const bool vm = L.c >= s, vp = L.c + s < L.Lc;
      const T al = vm ? -A / Bm : (T)0;
      const T ga = vp ? -C / Bp : (T)0;
      M.pl[(1 + 2 * r) * BS] = al;
      M.pl[(2 + 2 * r) * BS] = ga;
      const T An = vm ? al * Am : (T)0;
      const T Cn = vp ? ga * Cp : (T)0;
      B = B + (vm ? al * Cm : (T)0) + (vp ? ga * Ap : (T)0);
      A = An;
      C = Cn;
    }
  }
  M.pl[0] = (T)1 / B;
}

// z = M^-1 r for the chunk (padding entries of r must be zero).
template <int OPC, typename T, int K, int BS>
__device__ __forceinline__ void linepre_apply(const Lane<K>& L, const LineOp<OPC, T, K>& O,
                                              const LinePre<T, K>& M, const T (&r)[K],
                                              T (&z)[K]) {
  T y[K];
  y[0] = r[0];
  // interior unknowns k >= 1 have j > 0, so their lower coupling is the
  // operator's; a padding unknown's y never reaches a live one (its upper
  // coupling below is masked, and aL is zero in a partial chunk)
#pragma unroll
  for (int k = 1; k < K - 1; ++k) y[k] = r[k] - op_slo(O, k) * M.id[k - 1] * y[k - 1];
  y[K - 2] = y[K - 2] * M.id[K - 2];
#pragma unroll
  for (int k = K - 3; k >= 0; --k) {
    const T cu = (k + 1 < L.nval) ? op_sup(O, k) : (T)0;
    y[k] = (y[k] - cu * y[k + 1]) * M.id[k];
  }
  const T y0n = from_plus(y[0], 1, L.Lc);
  T R = r[K - 1] - M.aL * y[K - 2] - M.cL * y0n;
#pragma unroll
  for (int st = 0; st < kMaxPcr; ++st) {
    if (st < M.steps) {
      const int s = 1 << st;
      const T Rm = from_minus(R, s, L.Lc);
      const T Rp = from_plus(R, s, L.Lc);
      R = R + M.pl[(1 + 2 * st) * BS] * Rm + M.pl[(2 + 2 * st) * BS] * Rp;
    }
  }
  const T u = R * M.pl[0];
  T um = from_minus(u, 1, L.Lc);
  um = (L.c > 0) ? um : (T)0;
#pragma unroll
  for (int k = 0; k < K - 1; ++k) z[k] = y[k] - M.phi[k] * um - M.psi[k] * u;
  z[K - 1] = u;
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (k >= L.nval) z[k] = (T)0;
}


// ------------------------------------- preconditioner, constant coefficients
// HEAT: the chunk-interior factors are the same for all chunks of all lines
// (full chunks, and the last chunk of a line, which holds K - 1 unknowns
// when ns = 2^l - 1; a line of one chunk has ns < K unknowns in every lane)
// and the cyclic-reduction factors depend on the lane position c only, so
// they live in the work-group's HeatTab. A lane keeps four scalars: a0
// scales phiU (zero in the first chunk of a line), ps selects psiU (one in
// a full chunk), aL and cL are the couplings of its interface unknown.
template <typename T, int K>
struct LinePreH {
  const HeatTab<T, K>* h;
  T a0, ps, aL, cL;
  int steps;  // log2(Lc)
};

template <int OPC, typename T, int K>
using PreOf = typename std::conditional<OPC == OPC_HEAT, LinePreH<T, K>, LinePre<T, K>>::type;

// Builds the table's factors. Every thread of the work-group calls it after
// lineop_setup; it contains the barriers that publish the table. (The
// cyclic-reduction table arguments of the per-line preconditioner are not
// used: these factors live in the HeatTab.)
template <int OPC, typename T, int K, int BS>
__device__ __forceinline__ void linepre_setup(const Lane<K>& L, const LineOp<OPC_HEAT, T, K>& O,
                                              LinePreH<T, K>& M, T*, int, int*) {
  static_assert(OPC == OPC_HEAT, "constant-coefficient preconditioner");
  static_assert(K >= 2, "chunks hold at least two unknowns");
  HeatTab<T, K>* h = O.h;
  __syncthreads();  // weights visible
  if (threadIdx.x == 0) {
    // interior of a representative chunk: a full one, or the one chunk of
    // the line (thread 0 holds it) when Lc = 1
    const T dg = h->diag, sc = h->s;
    const int nrep = (L.Lc == 1) ? L.nval : K;
    T a[K], b[K], c[K], mm[K], id[K], cu[K], f[K], ph[K], ps[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      a[k] = (k > 0 && k < nrep) ? sc : (T)0;
      c[k] = (k + 1 < nrep) ? sc : (T)0;
      b[k] = (k < nrep) ? dg : (T)1;
    }
    mm[0] = (T)0;
    id[0] = (T)1 / b[0];
#pragma unroll
    for (int k = 1; k < K - 1; ++k) {
      mm[k] = a[k] * id[k - 1];
      id[k] = (T)1 / (b[k] - mm[k] * c[k - 1]);
    }
    mm[K - 1] = (T)0;
    id[K - 1] = (T)1;
#pragma unroll
    for (int k = 0; k < K; ++k) cu[k] = (k < K - 2) ? c[k] : (T)0;
    // phiU = T_I^-1 e_0, psiU = T_I^-1 (s e_{K-2})
    f[0] = (T)1;
#pragma unroll
    for (int k = 1; k < K - 1; ++k) f[k] = -mm[k] * f[k - 1];
    ph[K - 2] = f[K - 2] * id[K - 2];
#pragma unroll
    for (int k = K - 3; k >= 0; --k) ph[k] = (f[k] - cu[k] * ph[k + 1]) * id[k];
    ps[K - 2] = sc * id[K - 2];
#pragma unroll
    for (int k = K - 3; k >= 0; --k) ps[k] = -cu[k] * ps[k + 1] * id[k];
    ph[K - 1] = (T)0;
    ps[K - 1] = (T)0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      h->m[k] = mm[k];
      h->id[k] = id[k];
      h->cu[k] = cu[k];
      h->phiU[k] = ph[k];
      h->psiU[k] = ps[k];
    }
  }
  __syncthreads();  // interior factors visible
  const T sc = h->s;
  M.h = h;
  M.a0 = (L.nval > 0 && L.c > 0) ? sc : (T)0;
  M.ps = (L.nval == K) ? (T)1 : (T)0;
  M.aL = (L.nval == K) ? sc : (T)0;
  M.cL = L.nxt ? sc : (T)0;
  M.steps = 0;
  while ((1 << M.steps) < L.Lc) ++M.steps;
  if (threadIdx.x < 64) {
    // wave 0 holds line 0 in lanes 0..Lc-1: its interface system gives the
    // cyclic-reduction factors of every lane position
    const T bK = (K - 1 < L.nval) ? h->diag : (T)1;
    const T phi0n = from_plus(M.a0 * h->phiU[0], 1, L.Lc);
    const T psi0n = from_plus(M.ps * h->psiU[0], 1, L.Lc);
    T A = -M.aL * M.a0 * h->phiU[K - 2];
    T B = bK - M.aL * M.ps * h->psiU[K - 2] - M.cL * phi0n;
    T C = -M.cL * psi0n;
    const bool store = (L.line == 0);
#pragma unroll
    for (int r = 0; r < kMaxPcr; ++r) {
      const int s = 1 << r;
      if (s < L.Lc) {
        const T Am = from_minus(A, s, L.Lc), Bm = from_minus(B, s, L.Lc),
                Cm = from_minus(C, s, L.Lc);
        const T Ap = from_plus(A, s, L.Lc), Bp = from_plus(B, s, L.Lc),
                Cp = from_plus(C, s, L.Lc);
        const bool vm = L.c >= s, vp = L.c + s < L.Lc;
        const T al = vm ? -A / Bm : (T)0;
        const T ga = vp ? -C / Bp : (T)0;
        if (store) {
          h->pa[r][L.c] = al;
          h->pc[r][L.c] = ga;
        }
        const T An = vm ? al * Am : (T)0;
        const T Cn = vp ? ga * Cp : (T)0;
        B = B + (vm ? al * Cm : (T)0) + (vp ? ga * Ap : (T)0);
        A = An;
        C = Cn;
      }
    }
    if (store) h->pinv[L.c] = (T)1 / B;
  }
  __syncthreads();  // reduction factors visible
}

// z = M^-1 r for the chunk (padding entries of r must be zero).
template <int OPC, typename T, int K, int BS>
__device__ __forceinline__ void linepre_apply(const Lane<K>& L, const LineOp<OPC, T, K>&,
                                              const LinePreH<T, K>& M,
                                              const T (&r)[K], T (&z)[K]) {
  const HeatTab<T, K>* h = M.h;
  T y[K];
  y[0] = r[0];
#pragma unroll
  for (int k = 1; k < K - 1; ++k) y[k] = r[k] - h->m[k] * y[k - 1];
  y[K - 2] = y[K - 2] * h->id[K - 2];
#pragma unroll
  for (int k = K - 3; k >= 0; --k) y[k] = (y[k] - h->cu[k] * y[k + 1]) * h->id[k];
  const T y0n = from_plus(y[0], 1, L.Lc);
  T R = r[K - 1] - M.aL * y[K - 2] - M.cL * y0n;
#pragma unroll
  for (int st = 0; st < kMaxPcr; ++st) {
    if (st < M.steps) {
      const int s = 1 << st;
      const T Rm = from_minus(R, s, L.Lc);
      const T Rp = from_plus(R, s, L.Lc);
      R = R + h->pa[st][L.c] * Rm + h->pc[st][L.c] * Rp;
    }
  }
  const T u = R * h->pinv[L.c];
  T um = from_minus(u, 1, L.Lc);
  um = (L.c > 0) ? um : (T)0;
  const T ua = M.a0 * um, up = M.ps * u;
#pragma unroll
  for (int k = 0; k < K - 1; ++k) z[k] = y[k] - h->phiU[k] * ua - h->psiU[k] * up;
  z[K - 1] = u;
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (k >= L.nval) z[k] = (T)0;
}

}  // namespace ctm
