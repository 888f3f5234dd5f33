// Checks the wide solver's work-group placement (csrc/wide_map.h) on the
// host: for every launch shape gx x gy up to the given bounds, wide_map is a
// bijection of the blocks onto (block, task) pairs, and inside the groups of
// eight tasks every work-group whose linear id lands on XCD k (id mod 8 = k,
// the dispatcher's round robin) works on task k of its group; for every
// block count nb, wide_line_regroup is a bijection of [0, nb) and gives the
// blocks on one XCD consecutive virtual blocks. argv = max gx, max gy, max
// nb. Prints "ok" or the first failure.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "wide_map.h"

using namespace ctm;

int main(int argc, char** argv) {
  if (argc != 4) return 2;
  const int mgx = std::atoi(argv[1]), mgy = std::atoi(argv[2]), mnb = std::atoi(argv[3]);
  for (int gx = 1; gx <= mgx; ++gx)
    for (int gy = 1; gy <= mgy; ++gy) {
      std::vector<char> seen((size_t)gx * gy, 0);
      for (int by = 0; by < gy; ++by)
        for (int bx = 0; bx < gx; ++bx) {
          const WideBlock m = wide_map(bx, by, gx, gy);
          if (m.x < 0 || m.x >= gx || m.y < 0 || m.y >= gy) {
            std::printf("out of range gx=%d gy=%d bx=%d by=%d\n", gx, gy, bx, by);
            return 1;
          }
          char& s = seen[(size_t)m.y * gx + m.x];
          if (s) {
            std::printf("not injective gx=%d gy=%d bx=%d by=%d\n", gx, gy, bx, by);
            return 1;
          }
          s = 1;
          const long long lin = (long long)by * gx + bx;
          if (by < (gy & ~7) && (lin % 8) != (m.y % 8)) {
            std::printf("task off its XCD gx=%d gy=%d bx=%d by=%d\n", gx, gy, bx, by);
            return 1;
          }
          if (by >= (gy & ~7) && (m.x != bx || m.y != by)) {
            std::printf("last group not in plain order gx=%d gy=%d\n", gx, gy);
            return 1;
          }
        }
    }
  for (int nb = 0; nb <= mnb; ++nb) {
    std::vector<char> seen(nb, 0);
    const int q = nb / 8;
    for (int b = 0; b < nb; ++b) {
      const int v = wide_line_regroup(b, nb);
      if (v < 0 || v >= nb || seen[v]) {
        std::printf("regroup not a bijection nb=%d b=%d\n", nb, b);
        return 1;
      }
      seen[v] = 1;
      // blocks b and b + 8 (one XCD) take consecutive virtual blocks
      if (b + 8 < 8 * q && wide_line_regroup(b + 8, nb) != v + 1) {
        std::printf("regroup not consecutive nb=%d b=%d\n", nb, b);
        return 1;
      }
    }
  }
  std::printf("ok\n");
  return 0;
}
