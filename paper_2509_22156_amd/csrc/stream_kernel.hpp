// The streaming implicit-step kernel, for component grids that do not fit
// the on-chip solver (more than 8,192 unknowns, or lines longer than 512):
// one work-group of 1,024 threads per task (grid g, interval q), with every
// Krylov vector of the task in its own slot of an HBM scratch array. Thread
// t takes the points t, t + 1024, ... of the grid (canonical order, so every
// sweep is coalesced); a Krylov iteration is a few sweeps over the task's
// vectors, with block-wide reductions between them. FP64 throughout, CG or
// right-preconditioned BiCGStab (Section 4.1) with the same line-block
// preconditioner as the on-chip solver (exact solves of the stiff-axis
// lines, here one wave per line segment with 16 unknowns per lane and the
// factors kept in the task's scratch), the same vector roles as the on-chip
// chain kernel (ChainArgs).
//
// The stencil coefficients are evaluated per point and sweep from the grid
// descriptor and the coefficient tables in LDS; they match the on-chip
// operators of every class.
#pragma once

#include "line_layout.hpp"
#include "manufactured.hpp"

namespace ctm {

constexpr int kStreamThreads = 1024;
constexpr int kStreamW = kStreamThreads / 64;

// Scratch vectors of one task (each `sstride` doubles); SV_D holds the
// preconditioned direction in BiCGStab; SV_FM .. SV_FPSI the factors of the
// line preconditioner (stream_linepre_setup).
enum {
  SV_X = 0, SV_B, SV_R, SV_P, SV_Q, SV_RH, SV_S, SV_T, SV_D,
  SV_FM, SV_FID, SV_FCU, SV_FPHI, SV_FPSI, SV_N
};

// Coefficients of A = I + dt L at point p of grid g: the diagonal, and per
// axis the couplings to the lower and upper neighbour (zero where that
// neighbour is not an unknown), plus the point strides. D >= g.d bounds the
// dimension at compile time (2, 4 or 8), so that a low-dimensional grid
// keeps only its own axes in registers.
template <int OPC, int D>
struct PointCoef {
  double diag;
  double lo[D], up[D];
  int j[D];
};

template <int OPC, int D>
__device__ __forceinline__ void point_coef(const GridDev& g, const double* tl, double dt,
                                           double amp, int p, PointCoef<OPC, D>& c) {
  const int d = g.d;
  int rem = p;
#pragma unroll
  for (int i = D - 1; i >= 0; --i) {
    c.j[i] = 0;
    if (i < d) {
      c.j[i] = rem % g.n[i];
      rem /= g.n[i];
    }
  }
  double diag = 1.0;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    c.lo[i] = c.up[i] = 0.0;
    if (i >= d) continue;
    const int j = c.j[i];
    const int n = g.n[i];
    double lo = 0.0, up = 0.0;
    if constexpr (OPC == OPC_HEAT) {
      const double cc = dt * g.ih2[i];
      diag += 2.0 * cc;
      lo = up = -cc;
    } else if constexpr (OPC == OPC_SEP) {
      const double* t = tl + g.tab[i];  // Lo, D, Up of L, already times dt
      lo = t[j];
      diag += t[n + j];
      up = t[2 * n + j];
    } else if constexpr (OPC == OPC_VAR) {
      // a at the faces: 1 + amp * (face sine) * (node sines of the other axes)
      double es = 1.0;
#pragma unroll
      for (int k = 0; k < D; ++k)
        if (k < d && k != i) es *= tl[g.tab[k] + c.j[k]];
      const double* sm = tl + g.tab[i] + n;
      const double adn = 1.0 + amp * sm[j] * es, aup = 1.0 + amp * sm[j + 1] * es;
      const double cc = dt * g.ih2[i];
      diag += cc * (adn + aup);
      lo = -cc * adn;
      up = -cc * aup;
    } else {  // OPC_DRIFT: theta (d x d), then H (d)
      double w = 0.0;
#pragma unroll
      for (int k = 0; k < D; ++k)
        if (k < d) w += tl[i * d + k] * (g.lo[k] + (double)(c.j[k] + g.j0) * g.h[k]);
      // (reciprocals instead of divisions: the streaming kernels' stencil
      // sweeps are VALU-bound on this operator; 1/h is uniform per grid)
      const double h = g.h[i], half = tl[i * d + i] * 0.5 * h, H = tl[d * d + i];
      const double ih = 1.0 / h, ih2 = g.ih2[i];
      // central face fluxes w (u_j + u_{j+1}) / 2 (second order)
      const double wu = w + half, wd = w - half;
      diag += dt * (0.5 * (wu - wd) * ih + H * ih2);
      up = dt * (0.5 * wu * ih - 0.5 * H * ih2);
      lo = dt * (-0.5 * wd * ih - 0.5 * H * ih2);
    }
    c.lo[i] = (j > 0) ? lo : 0.0;
    c.up[i] = (j < n - 1) ? up : 0.0;
  }
  c.diag = diag;
}

// Neighbour indices of point p along axis i < D for the stencil: the point
// itself where the neighbour is not an unknown or the axis is past the
// grid's dimension (the coupling is zero there), computed without branches,
// so that every load is unconditional and the loads of a point issue
// together.
template <int OPC, int D>
__device__ __forceinline__ int stencil_lo(const GridDev& g, const PointCoef<OPC, D>& c, int i,
                                          int p) {
  const int has = (i < g.d) & (c.j[i] > 0);
  return p - has * g.stride[i];
}
template <int OPC, int D>
__device__ __forceinline__ int stencil_up(const GridDev& g, const PointCoef<OPC, D>& c, int i,
                                          int p) {
  const int has = (i < g.d) & (c.j[i] < g.n[i] - 1);
  return p + has * g.stride[i];
}

// y = A x at every point of the task; returns this thread's part of
// sum w[p] y[p] when w is given.
template <int OPC, int D>
__device__ __forceinline__ double stream_apply(const GridDev& g, const double* tl, double dt,
                                               double amp, const double* x, double* y,
                                               const double* w) {
  double acc = 0.0;
  for (int p = threadIdx.x; p < g.npts; p += kStreamThreads) {
    PointCoef<OPC, D> c;
    point_coef<OPC, D>(g, tl, dt, amp, p, c);
    double xl[D], xu[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
      xl[i] = x[stencil_lo(g, c, i, p)];
      xu[i] = x[stencil_up(g, c, i, p)];
    }
    double v = c.diag * x[p];
#pragma unroll
    for (int i = 0; i < D; ++i) v += c.lo[i] * xl[i] + c.up[i] * xu[i];
    y[p] = v;
    if (w) acc += w[p] * v;
  }
  return acc;
}

// ------------------------------------------------ line preconditioner
// M = the part of A that couples unknowns along the stiff axis (one
// tridiagonal block per line), as in the on-chip solver. A line of ns <=
// 1,024 unknowns is split into chunks of kSK consecutive unknowns, one
// chunk per lane of a segment of Lc = pow2ceil(ceil(ns / kSK)) <= 64 lanes
// of one wave; the waves of the work-group take the lines round by round.
// Per chunk: Thomas elimination of the first kSK-1 unknowns, whose
// responses to the neighbouring interface unknowns (phi, psi) are
// precomputed; the interface system (one unknown per lane, the chunk's
// last) is solved by parallel cyclic reduction over the segment's lanes;
// back-substitution. No barrier inside: a lane reads and writes only its own
// chunk, and neighbours come by cross-lane shuffles.
constexpr int kSK = 16;
static_assert(kSegLen == 64 * kSK, "a line segment is one wave of kSK-unknown chunks");

struct SLane {
  int line, c, Lc, j0, nval;
  bool nxt;        // the next chunk of the line holds unknowns
  long long base;  // canonical index of the line's first unknown
  int step;        // canonical stride along the stiff axis
};

// Unknowns of a line segment (the whole line when it is not cut) and the
// segments of the task (lines x segments per line).
__device__ __forceinline__ int stream_seg_len(const GridDev& g) {
  return g.nseg > 1 ? kSegLen : g.ns;
}
__device__ __forceinline__ int stream_segments(const GridDev& g) { return g.nlines * g.nseg; }

__device__ __forceinline__ int stream_line_rounds(const GridDev& g) {
  const int Lc = pow2ceil((stream_seg_len(g) + kSK - 1) / kSK);
  const int per_round = kStreamW * (64 / Lc);
  return (stream_segments(g) + per_round - 1) / per_round;
}

// Lane `lane` of wave `vwave` of the task: the wave holds 64 / Lc line
// segments, segments vwave * (64 / Lc) + lane / Lc. Segment index s is
// segment s / nlines of line s % nlines (segment-major), so consecutive
// indices are the same segment of neighbouring lines: neighbours in memory
// where the stiff axis is not the fastest. The first chunk of a segment is
// lane c = 0 and its last has no successor (nxt), so the line solve couples
// nothing across segments.
template <int D>
__device__ __forceinline__ void stream_lane_at(const GridDev& g, int vwave, int lane, SLane& L) {
  const int S = stream_seg_len(g);
  const int Lc = pow2ceil((S + kSK - 1) / kSK);
  L.Lc = Lc;
  L.c = lane & (Lc - 1);
  const int seg = vwave * (64 / Lc) + lane / Lc;
  const bool live = seg < stream_segments(g);
  const int sg = live ? seg / g.nlines : 0;
  L.line = live ? seg % g.nlines : g.nlines;
  const int s0 = sg * S;                               // first unknown of the segment
  const int s1 = s0 + S < g.ns ? s0 + S : g.ns;        // one past its last
  L.j0 = s0 + L.c * kSK;
  int nv = s1 - L.j0;
  nv = nv < 0 ? 0 : (nv > kSK ? kSK : nv);
  L.nval = live ? nv : 0;
  L.nxt = live && (L.j0 + kSK < s1);
  L.step = g.stride[g.sax];
  long long b = 0;
  const int rem = live ? L.line : 0;
#pragma unroll
  for (int m = 0; m < D - 1; ++m)
    if (m < g.d - 1) {
      const int ax = g.oax[m];
      b += (long long)((rem / g.lstride[m]) % g.n[ax]) * g.stride[ax];
    }
  L.base = b;
}

// The waves of the 1,024-thread work-group take the lines round by round.
template <int D>
__device__ __forceinline__ void stream_lane(const GridDev& g, int round, SLane& L) {
  const int t = threadIdx.x;
  stream_lane_at<D>(g, round * kStreamW + (t >> 6), t & 63, L);
}

// Stiff-axis couplings and diagonal of A at point p.
template <int OPC, int D>
__device__ __forceinline__ void line_coef(const GridDev& g, const double* tl, double dt,
                                          double amp, int p, double& lo, double& dg,
                                          double& up) {
  PointCoef<OPC, D> c;
  point_coef<OPC, D>(g, tl, dt, amp, p, c);
  lo = up = 0.0;  // (unrolled select: no dynamic register index)
#pragma unroll
  for (int ax = 0; ax < D; ++ax)
    if (ax == g.sax) {
      lo = c.lo[ax];
      up = c.up[ax];
    }
  dg = c.diag;
}

// Factors of M for the chunk of lane L, stored at the chunk's unknowns:
// FM = Thomas multipliers m_k (slot kSK-1: the diagonal of the interface
// unknown), FID = reciprocal pivots, FCU = upper couplings inside the
// chunk, FPHI/FPSI = responses of the eliminated unknowns to the previous
// and own interface unknown (slot kSK-1: the interface's couplings aL, cL).
// ftmp is a scratch vector (the forward spike). TF is the factors' storage
// type (the arithmetic is FP64): double here, float in the wide solver,
// whose slots then hold ss floats each.
template <int OPC, int D, typename TF = double>
__device__ __forceinline__ void linepre_setup_lane(const GridDev& g, const double* tl, double dt,
                                                   double amp, double* sv, long long ss,
                                                   double* ftmp, const SLane& L) {
  TF* FM = reinterpret_cast<TF*>(sv + SV_FM * ss);
  TF* FID = reinterpret_cast<TF*>(sv + SV_FID * ss);
  TF* FCU = reinterpret_cast<TF*>(sv + SV_FCU * ss);
  TF* FPHI = reinterpret_cast<TF*>(sv + SV_FPHI * ss);
  TF* FPSI = reinterpret_cast<TF*>(sv + SV_FPSI * ss);
  {
    // forward over the eliminated unknowns k = 0..kSK-2
    double idp = 0.0, cp = 0.0, fp = 0.0;
#pragma unroll 1
    for (int k = 0; k < kSK - 1; ++k) {
      const bool v = k < L.nval;
      const int j = L.j0 + k;
      const long long p = L.base + (long long)j * L.step;
      double lo = 0.0, dg = 1.0, up = 0.0;
      if (v) line_coef<OPC, D>(g, tl, dt, amp, (int)p, lo, dg, up);
      const double a = (v && j > 0) ? lo : 0.0;
      const double c = (v && k + 1 < L.nval) ? up : 0.0;
      const double b = v ? dg : 1.0;
      double m, id, f;
      if (k == 0) {
        m = 0.0;
        id = 1.0 / b;
        f = a;
      } else {
        m = a * idp;
        id = 1.0 / (b - m * cp);
        f = -m * fp;
      }
      if (v) {
        FM[p] = (TF)m;
        FID[p] = (TF)id;
        FCU[p] = (TF)((k < kSK - 2) ? c : 0.0);
        ftmp[p] = f;
      }
      idp = id;
      cp = c;
      fp = f;
    }
    // the interface unknown kSK-1 (present only in a full chunk)
    {
      const bool v = (L.nval == kSK);
      const long long p = L.base + (long long)(L.j0 + kSK - 1) * L.step;
      if (v) {
        double lo, dg, up;
        line_coef<OPC, D>(g, tl, dt, amp, (int)p, lo, dg, up);
        FM[p] = (TF)dg;
        FPHI[p] = (TF)lo;                      // aL (j0 + kSK - 1 > 0 always)
        FPSI[p] = (TF)(L.nxt ? up : 0.0);      // cL
      }
    }
    // backward: phi = T^-1 (a_0 e_0), psi = T^-1 (c_{kSK-2} e_{kSK-2})
    double php = 0.0, psp = 0.0;
#pragma unroll 1
    for (int k = kSK - 2; k >= 0; --k) {
      const bool v = k < L.nval;
      const long long p = L.base + (long long)(L.j0 + k) * L.step;
      double ph = 0.0, ps = 0.0;
      if (v) {
        const double id = (double)FID[p], f = ftmp[p];
        if (k == kSK - 2) {
          ph = f * id;
          ps = cp * id;  // c_{kSK-2}, from the forward pass
        } else {
          const double cu = (double)FCU[p];
          ph = (f - cu * php) * id;
          ps = -cu * psp * id;
        }
        FPHI[p] = (TF)ph;
        FPSI[p] = (TF)ps;
      }
      php = ph;
      psp = ps;
    }
  }
}

// The factors of every chunk of the task; called by every thread.
template <int OPC, int D>
__device__ void stream_linepre_setup(const GridDev& g, const double* tl, double dt, double amp,
                                     double* sv, long long ss, double* ftmp) {
  const int rounds = stream_line_rounds(g);
  for (int rd = 0; rd < rounds; ++rd) {
    SLane L;
    stream_lane<D>(g, rd, L);
    linepre_setup_lane<OPC, D>(g, tl, dt, amp, sv, ss, ftmp, L);
  }
}

// z = M^-1 r on every line of the task; returns this thread's part of
// sum w[p] z[p] when w is given. r must be complete on entry; ends with a
// barrier (z complete for the readers of neighbours). The eliminated
// unknowns' intermediate values go through z itself (a lane's chunk stays
// in the caches), so that no per-lane array competes for registers.
template <int D>
__device__ double stream_linepre_apply(const GridDev& g, const double* sv, long long ss,
                                       const double* r, double* z, const double* w) {
  const double* FM = sv + SV_FM * ss;
  const double* FID = sv + SV_FID * ss;
  const double* FCU = sv + SV_FCU * ss;
  const double* FPHI = sv + SV_FPHI * ss;
  const double* FPSI = sv + SV_FPSI * ss;
  const int rounds = stream_line_rounds(g);
  double acc = 0.0;
  for (int rd = 0; rd < rounds; ++rd) {
    SLane L;
    stream_lane<D>(g, rd, L);
    const bool full = (L.nval == kSK);
    const int ne = L.nval < kSK - 1 ? L.nval : kSK - 1;  // eliminated unknowns present
    const long long p0 = L.base + (long long)L.j0 * L.step;
    const long long st = L.step;
    // forward elimination: y_k = r_k - m_k y_{k-1}
    double y = 0.0, ylast = 0.0;
#pragma unroll 1
    for (int k = 0; k < ne; ++k) {
      const long long p = p0 + k * st;
      y = (k == 0) ? r[p] : r[p] - FM[p] * y;
      z[p] = y;
    }
    ylast = (ne == kSK - 1) ? y : 0.0;  // y_{kSK-2} before the back-substitution
    // back-substitution: y_k = (y_k - cu_k y_{k+1}) / pivot_k
    double yn = 0.0;
#pragma unroll 1
    for (int k = ne - 1; k >= 0; --k) {
      const long long p = p0 + k * st;
      yn = (k == kSK - 2) ? z[p] * FID[p] : (z[p] - FCU[p] * yn) * FID[p];
      z[p] = yn;
    }
    const double y0 = (ne > 0) ? yn : 0.0;
    const double y2 = (ne == kSK - 1) ? z[p0 + (kSK - 2) * st] : 0.0;
    (void)ylast;
    // interface equation of the chunk's last unknown u_c:
    //   A u_{c-1} + B u_c + C u_{c+1} = R
    const long long pl = p0 + (kSK - 1) * st;
    const long long p2 = p0 + (kSK - 2) * st;
    const double phi0 = (L.nval > 0) ? FPHI[p0] : 0.0, psi0 = (L.nval > 0) ? FPSI[p0] : 0.0;
    const double phi2 = (L.nval > kSK - 2) ? FPHI[p2] : 0.0;
    const double psi2 = (L.nval > kSK - 2) ? FPSI[p2] : 0.0;
    const double aL = full ? FPHI[pl] : 0.0, cL = full ? FPSI[pl] : 0.0;
    const double bL = full ? FM[pl] : 1.0;
    const double rL = full ? r[pl] : 0.0;
    const double phi0n = from_plus(phi0, 1, L.Lc), psi0n = from_plus(psi0, 1, L.Lc);
    const double y0n = from_plus(y0, 1, L.Lc);
    double A = -aL * phi2;
    double B = bL - aL * psi2 - cL * phi0n;
    double C = -cL * psi0n;
    double R = rL - aL * y2 - cL * y0n;
    // cyclic reduction over the lanes of the segment
#pragma unroll
    for (int sp = 0; sp < kMaxPcr; ++sp) {
      const int sh = 1 << sp;
      if (sh < L.Lc) {
        const double Am = from_minus(A, sh, L.Lc), Bm = from_minus(B, sh, L.Lc),
                     Cm = from_minus(C, sh, L.Lc), Rm = from_minus(R, sh, L.Lc);
        const double Ap = from_plus(A, sh, L.Lc), Bp = from_plus(B, sh, L.Lc),
                     Cp = from_plus(C, sh, L.Lc), Rp = from_plus(R, sh, L.Lc);
        const bool vm = L.c >= sh, vp = L.c + sh < L.Lc;
        const double al = vm ? -A / Bm : 0.0;
        const double ga = vp ? -C / Bp : 0.0;
        B = B + (vm ? al * Cm : 0.0) + (vp ? ga * Ap : 0.0);
        R = R + (vm ? al * Rm : 0.0) + (vp ? ga * Rp : 0.0);
        A = vm ? al * Am : 0.0;
        C = vp ? ga * Cp : 0.0;
      }
    }
    const double u = R / B;
    double um = from_minus(u, 1, L.Lc);
    um = (L.c > 0) ? um : 0.0;
    // z_k = y_k - phi_k u_{c-1} - psi_k u_c
#pragma unroll 1
    for (int k = 0; k < ne; ++k) {
      const long long p = p0 + k * st;
      const double zk = z[p] - FPHI[p] * um - FPSI[p] * u;
      z[p] = zk;
      if (w) acc += w[p] * zk;
    }
    if (full) {
      z[pl] = u;
      if (w) acc += w[pl] * u;
    }
  }
  __syncthreads();  // z complete for readers of other lanes' points
  return acc;
}

// ------------------------------------------------ Schwarz preconditioner
// The two-level overlapping Schwarz preconditioner of Section 2.1.2 on one
// task's grid (dense subdomain and coarse inverses computed at plan set-up,
// column-major, so that the threads of consecutive rows read consecutive
// addresses). cw: 3 * nbmax doubles of LDS.

// z (+)= C1 y: z_Omega_i += omega_i (R_i A R_i^T)^-1 y_Omega_i. The
// subdomains of one parity are disjoint (the overlap is at most half a
// subdomain), so each parity is one pass without write conflicts; the rows
// of a pass are spread over the work-group, nmax per subdomain. z must be
// set (zero) and y complete on entry; ends with a barrier.
__device__ __forceinline__ void schwarz_local(const SchwarzView& v, const SchwarzGrid& sg,
                                              const double* y, double* z) {
  const int nm = sg.nmax;
#pragma unroll 1
  for (int par = 0; par < 2; ++par) {
    const int nsp = (sg.nsub - par + 1) / 2;  // subdomains of this parity
    const long long rows = (long long)nsp * nm;
    for (long long f = threadIdx.x; f < rows; f += kStreamThreads) {
      const int k = par + 2 * (int)(f / nm);
      const int r = (int)(f % nm);
      const SchwarzSub& sb = v.sub[sg.sub0 + k];
      if (r >= sb.n) continue;
      const int* idx = v.ints + sb.idx;
      const double* M = v.linv + sb.inv;
      const int n = sb.n;
      double acc = 0.0;
#pragma unroll 4
      for (int c = 0; c < n; ++c) acc += M[(long long)c * n + r] * y[idx[c]];
      z[idx[r]] += sb.omega * acc;
    }
    __syncthreads();
  }
}

// wc[a] = (A_0^-1 R_0 y)_a in LDS (sums holds R_0 y on the way). y
// complete on entry; ends with a barrier.
__device__ __forceinline__ void schwarz_coarse(const SchwarzView& v, const SchwarzGrid& sg,
                                               const double* y, double* sums, double* wc) {
  const int nb = sg.nblk;
  const int* cord = v.ints + sg.cord;
  const int* bst = v.ints + sg.bst;
  for (int a = threadIdx.x; a < nb; a += kStreamThreads) {
    double sum = 0.0;
    for (int pos = bst[a]; pos < bst[a + 1]; ++pos) sum += y[cord[pos]];
    sums[a] = sum;
  }
  __syncthreads();
  const double* Mi = v.cinv + sg.cinv;
  for (int a = threadIdx.x; a < nb; a += kStreamThreads) {
    double acc = 0.0;
    for (int b = 0; b < nb; ++b) acc += Mi[(long long)b * nb + a] * sums[b];
    wc[a] = acc;
  }
  __syncthreads();
}

// z = C r: balanced G^T C1 G r + F r (G = I - A F; A symmetric, so G^T =
// I - F A) or additive C1 r + F r. Returns this thread's part of
// sum w[p] z[p] when w is given; ends with a barrier. The balanced form uses
// three scratch vectors of the task (the line preconditioner's factor
// slots, unused with this preconditioner). Out of line: the Krylov loops
// that call it stay small enough to be inlined into the kernel.
template <int OPC, int D>
__device__ __noinline__ double schwarz_apply(const GridDev& g, const double* tl, double dt,
                                             double amp, const SchwarzView& v,
                                             const SchwarzGrid& sg, double* cw, double* sv,
                                             long long ss, const double* r, double* z,
                                             const double* w) {
  const int np = g.npts;
  const int* cblk = v.ints + sg.cblk;
  double* c0 = cw;                  // A_0^-1 R_0 r
  double* c1 = cw + v.nbmax;        // block sums of a coarse solve
  double* c2 = cw + 2 * v.nbmax;    // A_0^-1 R_0 A C1 G r (balanced)
  double acc = 0.0;
  if (v.balanced) {
    double* T = sv + SV_FM * ss;   // F r
    double* U = sv + SV_FID * ss;  // G r = r - A F r
    double* Y = sv + SV_FCU * ss;  // A C1 G r
    schwarz_coarse(v, sg, r, c1, c0);
    for (int p = threadIdx.x; p < np; p += kStreamThreads) T[p] = c0[cblk[p]];
    __syncthreads();
    stream_apply<OPC, D>(g, tl, dt, amp, T, U, nullptr);
    for (int p = threadIdx.x; p < np; p += kStreamThreads) {
      U[p] = r[p] - U[p];
      z[p] = 0.0;
    }
    __syncthreads();
    schwarz_local(v, sg, U, z);
    stream_apply<OPC, D>(g, tl, dt, amp, z, Y, nullptr);
    __syncthreads();
    schwarz_coarse(v, sg, Y, c1, c2);  // A_0^-1 R_0 A C1 G r; c0 (for F r) stays
    for (int p = threadIdx.x; p < np; p += kStreamThreads) {
      const int b = cblk[p];
      const double zp = z[p] - c2[b] + c0[b];
      z[p] = zp;
      if (w) acc += w[p] * zp;
    }
  } else {
    schwarz_coarse(v, sg, r, c1, c0);
    for (int p = threadIdx.x; p < np; p += kStreamThreads) z[p] = 0.0;
    __syncthreads();
    schwarz_local(v, sg, r, z);
    for (int p = threadIdx.x; p < np; p += kStreamThreads) {
      const double zp = z[p] + c0[cblk[p]];
      z[p] = zp;
      if (w) acc += w[p] * zp;
    }
  }
  __syncthreads();
  return acc;
}

// The task's preconditioner: Schwarz when the launch carries it (sg), else
// the line-block solve. Same contract as stream_linepre_apply.
template <int OPC, int D>
__device__ __forceinline__ double stream_precond(const GridDev& g, const double* tl,
                                                 const ChainArgs& a, const SchwarzGrid* sg,
                                                 double* cw, double* sv, long long ss,
                                                 const double* r, double* z, const double* w) {
  if (sg) return schwarz_apply<OPC, D>(g, tl, a.dt, a.amp, a.sch, *sg, cw, sv, ss, r, z, w);
  return stream_linepre_apply<D>(g, sv, ss, r, z, w);
}

// One implicit step: x <- (I + dt L)^-1 b, x holding the initial guess.
// Preconditioned CG (symmetric operators).
template <int OPC, int D>
__device__ int stream_cg(const GridDev& g, const double* tl, const ChainArgs& a, double* sv,
                         long long ss, RedRing& ring, double tol2, int* flag, double* rr0,
                         const SchwarzGrid* sg, double* cw) {
  double* X = sv + SV_X * ss;
  double* B = sv + SV_B * ss;
  double* R = sv + SV_R * ss;
  double* P = sv + SV_P * ss;
  double* Q = sv + SV_Q * ss;
  double* Z = sv + SV_S * ss;
  const int np = g.npts;
  stream_apply<OPC, D>(g, tl, a.dt, a.amp, X, Q, nullptr);
  double s0[2] = {0.0, 0.0};  // (r, r), (b, b)
  for (int p = threadIdx.x; p < np; p += kStreamThreads) {
    const double r = B[p] - Q[p];
    R[p] = r;
    s0[0] += r * r;
    s0[1] += B[p] * B[p];
  }
  block_sum<kStreamW, 2, double>(s0, ring);  // also orders R before the preconditioner
  const double bb = s0[1];
  if (!(s0[0] == s0[0]) || !(bb == bb)) {
    *flag |= FLAG_NONFINITE;
    return 0;
  }
  *rr0 = s0[0];  // the initial residual (residual mode's F-step norm)
  if (s0[0] <= tol2 * bb) return 0;
  double rz1[1] = {stream_precond<OPC, D>(g, tl, a, sg, cw, sv, ss, R, Z, R)};
  block_sum<kStreamW, 1, double>(rz1, ring);
  double rz = rz1[0];
  for (int p = threadIdx.x; p < np; p += kStreamThreads) P[p] = Z[p];
  __syncthreads();
  for (int it = 1; it <= a.maxit; ++it) {
    double pq[1] = {stream_apply<OPC, D>(g, tl, a.dt, a.amp, P, Q, P)};
    block_sum<kStreamW, 1, double>(pq, ring);
    if (!(pq[0] != 0.0) || !(pq[0] == pq[0])) {
      *flag |= (pq[0] == pq[0]) ? FLAG_BREAKDOWN : FLAG_NONFINITE;
      return it;
    }
    const double alpha = rz / pq[0];
    double s1[1] = {0.0};
    for (int p = threadIdx.x; p < np; p += kStreamThreads) {
      X[p] += alpha * P[p];
      const double r = R[p] - alpha * Q[p];
      R[p] = r;
      s1[0] += r * r;
    }
    block_sum<kStreamW, 1, double>(s1, ring);
    if (!(s1[0] == s1[0])) {
      *flag |= FLAG_NONFINITE;
      return it;
    }
    if (s1[0] <= tol2 * bb) return it;
    double rzn[1] = {stream_precond<OPC, D>(g, tl, a, sg, cw, sv, ss, R, Z, R)};
    block_sum<kStreamW, 1, double>(rzn, ring);
    const double beta = rzn[0] / rz;
    rz = rzn[0];
    for (int p = threadIdx.x; p < np; p += kStreamThreads) P[p] = Z[p] + beta * P[p];
    __syncthreads();  // P complete before the next apply reads neighbours
  }
  *flag |= FLAG_NOCONV;
  return a.maxit;
}

// Right-preconditioned BiCGStab (van der Vorst): p^ = M^-1 p, v = A p^,
// s^ = M^-1 s, t = A s^, x += alpha p^ + omega s^ (the first part as soon as
// alpha is known, so that p^ and s^ share one scratch vector).
template <int OPC, int D>
__device__ int stream_bicgstab(const GridDev& g, const double* tl, const ChainArgs& a,
                               double* sv, long long ss, RedRing& ring, double tol2,
                               int* flag, double* rr0, const SchwarzGrid* sg, double* cw) {
  double* X = sv + SV_X * ss;
  double* B = sv + SV_B * ss;
  double* R = sv + SV_R * ss;
  double* P = sv + SV_P * ss;
  double* V = sv + SV_Q * ss;
  double* RH = sv + SV_RH * ss;
  double* S = sv + SV_S * ss;
  double* T = sv + SV_T * ss;
  double* H = sv + SV_D * ss;  // p^, then s^
  const int np = g.npts;
  stream_apply<OPC, D>(g, tl, a.dt, a.amp, X, V, nullptr);
  double s0[2] = {0.0, 0.0};
  for (int p = threadIdx.x; p < np; p += kStreamThreads) {
    const double r = B[p] - V[p];
    R[p] = r;
    RH[p] = r;
    P[p] = r;
    s0[0] += r * r;
    s0[1] += B[p] * B[p];
  }
  block_sum<kStreamW, 2, double>(s0, ring);
  const double bb = s0[1];
  if (!(s0[0] == s0[0]) || !(bb == bb)) {
    *flag |= FLAG_NONFINITE;
    return 0;
  }
  *rr0 = s0[0];  // the initial residual (residual mode's F-step norm)
  if (s0[0] <= tol2 * bb) return 0;
  double rho = s0[0];
  for (int it = 1; it <= a.maxit; ++it) {
    stream_precond<OPC, D>(g, tl, a, sg, cw, sv, ss, P, H, nullptr);
    double s2[1] = {stream_apply<OPC, D>(g, tl, a.dt, a.amp, H, V, RH)};
    block_sum<kStreamW, 1, double>(s2, ring);
    if (!(s2[0] != 0.0) || !(s2[0] == s2[0])) {
      *flag |= (s2[0] == s2[0]) ? FLAG_BREAKDOWN : FLAG_NONFINITE;
      return it;
    }
    const double alpha = rho / s2[0];
    for (int p = threadIdx.x; p < np; p += kStreamThreads) {
      X[p] += alpha * H[p];
      S[p] = R[p] - alpha * V[p];
    }
    __syncthreads();  // S complete before the preconditioner reads whole lines
    stream_precond<OPC, D>(g, tl, a, sg, cw, sv, ss, S, H, nullptr);
    double s3[3] = {0.0, 0.0, 0.0};  // (t, s), (t, t), (s, s)
    for (int p = threadIdx.x; p < np; p += kStreamThreads) {
      PointCoef<OPC, D> c;
      point_coef<OPC, D>(g, tl, a.dt, a.amp, p, c);
      double hl[D], hu[D];
#pragma unroll
      for (int i = 0; i < D; ++i) {
        hl[i] = H[stencil_lo(g, c, i, p)];
        hu[i] = H[stencil_up(g, c, i, p)];
      }
      double v = c.diag * H[p];
#pragma unroll
      for (int i = 0; i < D; ++i) v += c.lo[i] * hl[i] + c.up[i] * hu[i];
      T[p] = v;
      s3[0] += v * S[p];
      s3[1] += v * v;
      s3[2] += S[p] * S[p];
    }
    block_sum<kStreamW, 3, double>(s3, ring);
    if (s3[2] <= tol2 * bb) return it;  // x already holds x + alpha p^
    if (!(s3[1] != 0.0) || !(s3[1] == s3[1])) {
      *flag |= (s3[1] == s3[1]) ? FLAG_BREAKDOWN : FLAG_NONFINITE;
      return it;
    }
    const double omega = s3[0] / s3[1];
    double s4[2] = {0.0, 0.0};  // (r, r), (rh, r)
    for (int p = threadIdx.x; p < np; p += kStreamThreads) {
      X[p] += omega * H[p];
      const double r = S[p] - omega * T[p];
      R[p] = r;
      s4[0] += r * r;
      s4[1] += RH[p] * r;
    }
    block_sum<kStreamW, 2, double>(s4, ring);
    if (!(s4[0] == s4[0])) {
      *flag |= FLAG_NONFINITE;
      return it;
    }
    if (s4[0] <= tol2 * bb) return it;
    if (s4[1] == 0.0 || omega == 0.0) {
      *flag |= FLAG_BREAKDOWN;
      return it;
    }
    const double beta = (s4[1] / rho) * (alpha / omega);
    rho = s4[1];
    for (int p = threadIdx.x; p < np; p += kStreamThreads)
      P[p] = R[p] + beta * (P[p] - omega * V[p]);
    __syncthreads();  // P complete before the preconditioner reads whole lines
  }
  *flag |= FLAG_NOCONV;
  return a.maxit;
}

// Scratch of task t of the launch: sv = scratch + t * SV_N * ss.
template <int OPC, int SOLVER, int D>
__global__ void __launch_bounds__(kStreamThreads)
    stream_kernel(ChainArgs a, int tabmax, double* scratch, long long ss) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ GridDev gs;
  __shared__ double red[2 * 64];
  if (a.skip && *a.skip != 0.0) return;  // whole work-group: queued past convergence
  double* tl = reinterpret_cast<double*>(smem);
  const int2 task = a.tasks[blockIdx.x];
  const int q = task.y;
  {
    const int* src = reinterpret_cast<const int*>(a.grids + task.x);
    int* dst = reinterpret_cast<int*>(&gs);
    for (int t = threadIdx.x; t < (int)(sizeof(GridDev) / sizeof(int)); t += kStreamThreads)
      dst[t] = src[t];
  }
  __syncthreads();
  const GridDev& g = gs;
  load_tables<OPC, double, kStreamThreads>(g, a.tab64, a.dt, tl);
  __syncthreads();
  double* sv = scratch + (long long)blockIdx.x * SV_N * ss;
  double* X = sv + SV_X * ss;
  double* B = sv + SV_B * ss;
  const int np = g.npts;
  const long long off = g.off;
  auto at = [&](const VecRef& r, long long idx) { return r.base + idx * a.slen + off; };
  const double* st = a.start.base ? at(a.start, a.start.a * q + a.start.b) : nullptr;
  double* wb = a.start_wb.base ? at(a.start_wb, a.start_wb.a * q + a.start_wb.b) : nullptr;
  for (int p = threadIdx.x; p < np; p += kStreamThreads) {
    const double v = st ? st[p] : 0.0;
    B[p] = v;
    if (wb) wb[p] = v;
  }
  // the Schwarz preconditioner (its LDS after the tables), or the line
  // preconditioner's factors, once per chain (each lane later reads only
  // what it wrote here)
  const SchwarzGrid* sg = a.sch.grid ? a.sch.grid + task.x : nullptr;
  double* cw = tl + tabmax;
  if (!sg) stream_linepre_setup<OPC, D>(g, tl, a.dt, a.amp, sv, ss, sv + SV_S * ss);
  __syncthreads();
  RedRing ring{red, 0};
  int flag = 0;
  long long kr_sum = 0, kr_max = 0;
  const double tol2 = a.tol * a.tol;
  // residual mode (as in the on-chip kernel): fixed-count steps from the
  // previous iterate, the forcing before the step, and the exact space-time
  // residual rho = v - A target in place of the last step
  const bool res = a.resmode != 0;
  double res_max = 0.0;
  bool have_rho = false;
  for (int j = 1; j <= a.nsteps; ++j) {
    const bool last = (j == a.nsteps);
    const double* f = a.forcing.base ? at(a.forcing, a.forcing.a * q + a.forcing.b + j) : nullptr;
    double* is = (a.inter.base && j < a.nsteps) ? at(a.inter, a.inter.a * q + a.inter.b + j)
                                                 : nullptr;
    if (res && f) {
      for (int p = threadIdx.x; p < np; p += kStreamThreads) B[p] += f[p];
      __syncthreads();
    }
    if (res && last && a.target.base) {
      const double* tg = at(a.target, a.target.a * q + a.target.b);
      double* Q = sv + SV_Q * ss;
      stream_apply<OPC, D>(g, tl, a.dt, a.amp, tg, Q, nullptr);
      __syncthreads();
      for (int p = threadIdx.x; p < np; p += kStreamThreads) B[p] -= Q[p];
      __syncthreads();
      have_rho = true;
      break;
    }
    const VecRef gr = last ? a.guess_fin : a.guess;
    const double* gx = gr.base ? at(gr, gr.a * q + gr.b + (last ? 0 : j)) : nullptr;
    // manufactured heat problem: the step solves (I + dt L) x = v + dt f(t_j)
    // (the guess taken before the forcing is added, as on chip)
    const bool mms = (OPC == OPC_HEAT) && a.fkind && !res;
    const double tj = a.ft0 + (double)q * a.ftq + (double)j * a.dt;
    for (int p = threadIdx.x; p < np; p += kStreamThreads) {
      X[p] = gx ? gx[p] : B[p];
      if (mms) B[p] += a.dt * mms_point<D>(g, p, tj);
    }
    __syncthreads();
    int it;
    double r0 = 0.0;
    if constexpr (SOLVER == SOLV_CG)
      it = stream_cg<OPC, D>(g, tl, a, sv, ss, ring, tol2, &flag, &r0, sg, cw);
    else
      it = stream_bicgstab<OPC, D>(g, tl, a, sv, ss, ring, tol2, &flag, &r0, sg, cw);
    if (res) {
      flag &= ~(FLAG_NOCONV | FLAG_BREAKDOWN);
      res_max = r0 > res_max ? r0 : res_max;
    }
    kr_sum += it;
    kr_max = it > kr_max ? it : kr_max;
    __syncthreads();  // every thread's X final
    for (int p = threadIdx.x; p < np; p += kStreamThreads) {
      const double v = X[p] + ((f && !res) ? f[p] : 0.0);
      B[p] = v;
      if (is) is[p] = v;
    }
    __syncthreads();
  }
  if (a.fin.base) {
    double* dst = at(a.fin, a.fin.a * q + a.fin.b);
    const double* tg = (a.target.base && !have_rho) ? at(a.target, a.target.a * q + a.target.b)
                                                     : nullptr;
    double rr[1] = {0.0};
    for (int p = threadIdx.x; p < np; p += kStreamThreads) {
      const double v = tg ? B[p] - tg[p] : B[p];
      dst[p] = v;
      rr[0] += v * v;
    }
    if (a.target.base) {
      block_sum<kStreamW, 1, double>(rr, ring);
      if (res) rr[0] = rr[0] > res_max ? rr[0] : res_max;
      if (threadIdx.x == 0 && a.res2) a.res2[blockIdx.x] = rr[0];
    }
  }
  if (threadIdx.x == 0) {
    if (a.counters) {
      atomicAdd(&a.counters[CNT_KRYLOV], (unsigned long long)kr_sum);
      atomicMax(&a.counters[CNT_KRYLOV_MAX], (unsigned long long)kr_max);
      atomicAdd(&a.counters[CNT_SOLVES], (unsigned long long)a.nsteps);
      atomicAdd(&a.counters[CNT_WORK], (unsigned long long)kr_sum * (unsigned long long)np);
      atomicAdd(&a.counters[CNT_DOFSTEPS], (unsigned long long)a.nsteps * (unsigned long long)np);
    }
    if (flag && a.status) atomicOr(a.status, flag);
  }
}

template <int OPC, int SOLVER, int D>
hipError_t launch_stream_t(const ChainArgs& a, int ntasks, int tabmax, double* scratch,
                           long long ss, hipStream_t s) {
  if (ntasks <= 0) return hipSuccess;
  // the coefficient tables, then the Schwarz preconditioner's coarse vectors
  const size_t smem =
      ((size_t)tabmax + (a.sch.grid ? 3 * (size_t)a.sch.nbmax : 0)) * sizeof(double);
  hipLaunchKernelGGL((stream_kernel<OPC, SOLVER, D>), dim3(ntasks), dim3(kStreamThreads), smem, s,
                     a, tabmax, scratch, ss);
  return hipGetLastError();
}

// y = (I + dt L) x on every grid, point-wise (one work-group per grid); the
// standalone apply for plans with streaming grids.
template <int OPC, int D>
__global__ void __launch_bounds__(kStreamThreads)
    stream_apply_kernel(const GridDev* __restrict__ grids, const double* __restrict__ tab64,
                        double amp, double dt, const double* __restrict__ x,
                        double* __restrict__ y) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ GridDev gs;
  double* tl = reinterpret_cast<double*>(smem);
  {
    const int* src = reinterpret_cast<const int*>(grids + blockIdx.x);
    int* dst = reinterpret_cast<int*>(&gs);
    for (int t = threadIdx.x; t < (int)(sizeof(GridDev) / sizeof(int)); t += kStreamThreads)
      dst[t] = src[t];
  }
  __syncthreads();
  load_tables<OPC, double, kStreamThreads>(gs, tab64, dt, tl);
  __syncthreads();
  stream_apply<OPC, D>(gs, tl, dt, amp, x + gs.off, y + gs.off, nullptr);
}

}  // namespace ctm
