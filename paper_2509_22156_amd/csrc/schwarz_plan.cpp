// Host part of the two-level overlapping Schwarz preconditioner (Section
// 2.1.2): the Hilbert-curve order of a grid's unknowns, the disjoint
// partition along the curve, the overlap and its weights, and the coarse
// blocks. The dense subdomain and coarse inverses are computed on the
// device (schwarz_ops.hip).
#include <algorithm>
#include <cstring>
#include <numeric>

#include "ctm_internal.h"

namespace ctm {

namespace {

// Index along the d-dimensional Hilbert curve of order `bits` of the lattice
// point x (coordinates in [0, 2^bits)), after J. Skilling, "Programming the
// Hilbert curve" (AIP Conf. Proc. 707, 2004): the coordinates are turned
// into the curve's transposed index (undo of the reflections and exchanges
// from the most significant bit down, then Gray encoding), whose bits, read
// interleaved from the top, form the index. Up to 6 x 20 bits: 128-bit key.
unsigned __int128 hilbert_key(const int* x_in, int d, int bits) {
  unsigned X[MAXD];
  for (int i = 0; i < d; ++i) X[i] = (unsigned)x_in[i];
  if (bits <= 0 || d <= 0) return 0;
  const unsigned M = 1u << (bits - 1);
  for (unsigned Q = M; Q > 1; Q >>= 1) {
    const unsigned P = Q - 1;
    for (int i = 0; i < d; ++i) {
      if (X[i] & Q) {
        X[0] ^= P;
      } else {
        const unsigned t = (X[0] ^ X[i]) & P;
        X[0] ^= t;
        X[i] ^= t;
      }
    }
  }
  for (int i = 1; i < d; ++i) X[i] ^= X[i - 1];
  unsigned t = 0;
  for (unsigned Q = M; Q > 1; Q >>= 1)
    if (X[d - 1] & Q) t ^= Q - 1;
  for (int i = 0; i < d; ++i) X[i] ^= t;
  unsigned __int128 h = 0;
  for (int b = bits - 1; b >= 0; --b)
    for (int i = 0; i < d; ++i) h = (h << 1) | ((X[i] >> b) & 1u);
  return h;
}

}  // namespace

bool schwarz_decompose(const GridDev& gd, int S, SchwarzGrid& sg, std::vector<SchwarzSub>& subs,
                       std::vector<int>& ints, long long& linv_len, long long& cinv_len,
                       std::string& msg) {
  const int d = gd.d;
  const int N = gd.npts;
  int lmax = 0;
  for (int i = 0; i < d; ++i) lmax = std::max(lmax, gd.lev[i]);
  // lattice coordinates with virtual nodes: unknown J of axis i at J 2^(lmax - l_i)
  std::vector<unsigned __int128> key(N);
  int x[MAXD];
  for (int p = 0; p < N; ++p) {
    int rem = p;
    for (int i = d - 1; i >= 0; --i) {
      const int j = rem % gd.n[i];
      rem /= gd.n[i];
      x[i] = (j + gd.j0) << (lmax - gd.lev[i]);
    }
    key[p] = hilbert_key(x, d, lmax);
  }
  std::vector<int> order(N);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return key[a] < key[b]; });

  // disjoint partition: P = ceil(N / 2^S), the N - P w larger ones first
  const long long cap = 1LL << S;
  const int P = (int)std::max<long long>(1, (N + cap - 1) / cap);
  const int w = N / P;
  const int big = N - P * w;
  std::vector<int> start(P + 1, 0);
  for (int i = 0; i < P; ++i) start[i + 1] = start[i] + (i < big ? w + 1 : w);
  // overlap floor(gamma w) with gamma = 1/2
  const int ov = (P > 1) ? w / 2 : 0;
  std::vector<int> mult(N, 0);
  std::vector<int> ea(P), eb(P);
  int nmax = 0;
  for (int i = 0; i < P; ++i) {
    ea[i] = std::max(0, start[i] - ov);
    eb[i] = std::min(N, start[i + 1] + ov);
    for (int k = ea[i]; k < eb[i]; ++k) ++mult[k];
    nmax = std::max(nmax, eb[i] - ea[i]);
  }
  // coarse blocks: q per disjoint subdomain (at most its size)
  const int q = (S >= 4) ? (1 << (S - 4)) : 1;
  std::vector<int> bst;
  for (int i = 0; i < P; ++i) {
    const int n = start[i + 1] - start[i];
    const int nb = std::min(q, n);
    const int bw = n / nb, bbig = n - nb * bw;
    int cur = start[i];
    for (int b = 0; b < nb; ++b) {
      bst.push_back(cur);
      cur += (b < bbig) ? bw + 1 : bw;
    }
  }
  const int nblk = (int)bst.size();
  bst.push_back(N);
  if (nblk > kSchwarzMaxBlocks) {
    msg = "Schwarz preconditioner: a grid of " + std::to_string(N) + " unknowns has " +
          std::to_string(nblk) + " coarse blocks (at most " +
          std::to_string(kSchwarzMaxBlocks) + ")";
    return false;
  }

  sg.nsub = P;
  sg.nblk = nblk;
  sg.nmax = nmax;
  sg.sub0 = (long long)subs.size();
  sg.cinv = cinv_len;
  cinv_len += (long long)nblk * nblk;
  sg.cord = (long long)ints.size();
  ints.insert(ints.end(), order.begin(), order.end());
  sg.cblk = (long long)ints.size();
  {
    std::vector<int> cb(N, 0);
    for (int b = 0; b < nblk; ++b)
      for (int pos = bst[b]; pos < bst[b + 1]; ++pos) cb[order[pos]] = b;
    ints.insert(ints.end(), cb.begin(), cb.end());
  }
  sg.bst = (long long)ints.size();
  ints.insert(ints.end(), bst.begin(), bst.end());
  for (int i = 0; i < P; ++i) {
    SchwarzSub sb;
    std::memset(&sb, 0, sizeof(sb));
    sb.n = eb[i] - ea[i];
    int mm = 0;
    for (int k = start[i]; k < start[i + 1]; ++k) mm = std::max(mm, mult[k]);
    sb.omega = 1.0 / (double)mm;
    sb.idx = (long long)ints.size();
    ints.insert(ints.end(), order.begin() + ea[i], order.begin() + eb[i]);
    std::vector<std::pair<int, int>> pr(sb.n);
    for (int r = 0; r < sb.n; ++r) pr[r] = {order[ea[i] + r], r};
    std::sort(pr.begin(), pr.end());
    sb.srt = (long long)ints.size();
    for (const auto& e : pr) {
      ints.push_back(e.first);
      ints.push_back(e.second);
    }
    sb.inv = linv_len;
    linv_len += (long long)sb.n * sb.n;
    subs.push_back(sb);
  }
  return true;
}

}  // namespace ctm
