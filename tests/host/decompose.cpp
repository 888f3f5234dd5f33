// Prints the library's Schwarz decomposition of one grid (host code of
// csrc/schwarz_plan.cpp) for comparison with the oracle: argv = d j0 S l_1
// .. l_d. Output lines: "order ...", "blocks ...", then one "sub n omega
// points..." line per subdomain, "pairs ok" when every subdomain's sorted
// (point, row) pairs agree with its point list.
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "ctm_internal.h"

using namespace ctm;

int main(int argc, char** argv) {
  if (argc < 4) return 2;
  const int d = std::atoi(argv[1]);
  if (d < 1 || d > MAXD || argc != 4 + d) return 2;
  GridDev gd;
  std::memset(&gd, 0, sizeof(gd));
  gd.d = d;
  gd.j0 = std::atoi(argv[2]);
  const int S = std::atoi(argv[3]);
  long long np = 1;
  for (int i = 0; i < d; ++i) {
    gd.lev[i] = std::atoi(argv[4 + i]);
    gd.n[i] = gd.j0 ? (1 << gd.lev[i]) - 1 : (1 << gd.lev[i]);
    np *= gd.n[i];
  }
  gd.npts = (int)np;
  SchwarzGrid sg;
  std::memset(&sg, 0, sizeof(sg));
  std::vector<SchwarzSub> subs;
  std::vector<int> ints;
  long long linv = 0, cinv = 0;
  std::string msg;
  if (!schwarz_decompose(gd, S, sg, subs, ints, linv, cinv, msg)) {
    std::printf("error %s\n", msg.c_str());
    return 0;
  }
  std::printf("order");
  for (int p = 0; p < gd.npts; ++p) std::printf(" %d", ints[sg.cord + p]);
  std::printf("\nblocks");
  for (int b = 0; b <= sg.nblk; ++b) std::printf(" %d", ints[sg.bst + b]);
  std::printf("\n");
  bool pairs = true;
  long long lsum = 0;
  for (int k = 0; k < sg.nsub; ++k) {
    const SchwarzSub& sb = subs[sg.sub0 + k];
    std::printf("sub %d %.17g", sb.n, sb.omega);
    for (int r = 0; r < sb.n; ++r) std::printf(" %d", ints[sb.idx + r]);
    std::printf("\n");
    for (int m = 0; m < sb.n; ++m) {
      const int pt = ints[sb.srt + 2 * m], row = ints[sb.srt + 2 * m + 1];
      if (row < 0 || row >= sb.n || ints[sb.idx + row] != pt) pairs = false;
      if (m > 0 && ints[sb.srt + 2 * (m - 1)] >= pt) pairs = false;
    }
    if (sb.inv != lsum) pairs = false;
    lsum += (long long)sb.n * sb.n;
  }
  for (int p = 0; p < gd.npts; ++p) {
    const int b = ints[sg.cblk + p];
    bool in = false;
    for (int pos = ints[sg.bst + b]; pos < ints[sg.bst + b + 1]; ++pos)
      in |= (ints[sg.cord + pos] == p);
    if (!in) pairs = false;
  }
  if (cinv != (long long)sg.nblk * sg.nblk || linv != lsum) pairs = false;
  std::printf(pairs ? "pairs ok\n" : "pairs bad\n");
  return 0;
}
