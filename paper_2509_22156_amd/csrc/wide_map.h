// Work-group placement of the wide streaming solver: which (block, task)
// pair a work-group of a launch works on. Plain integer functions, shared by
// the kernels (wide_kernel.hpp) and the host test of the mapping.
//
// The dispatcher deals a launch's work-groups to the eight XCDs of the GPU
// round robin in linear order (y * gx + x for a gx x gy grid), and each XCD
// has its own L2. wide_map takes the tasks in groups of eight: the eight
// gx-block rows of a group form one range of linear ids, a multiple of eight
// long, and the ids of that range on XCD k all become blocks of task k of the
// group (block = position among them), so a task runs on one XCD. A last
// group of fewer than eight tasks keeps the plain order. wide_line_regroup
// serves that last group: block b of a task's nb line blocks becomes virtual
// block (b mod 8) q + b / 8 with q = nb / 8, so that the blocks on one XCD
// (b, b + 8, ...) take q consecutive virtual blocks; blocks from 8 q on keep
// their index. Both are bijections.
#pragma once

#include <hip/hip_runtime.h>

namespace ctm {

struct WideBlock {
  int x, y;  // block of the task, task
};

__host__ __device__ inline bool wide_in_group(unsigned by, unsigned gy) {
  return by < (gy & ~7u);
}

__host__ __device__ inline WideBlock wide_map(unsigned bx, unsigned by, unsigned gx,
                                              unsigned gy) {
  if (!wide_in_group(by, gy)) return WideBlock{(int)bx, (int)by};
  const unsigned off = (by & 7u) * gx + bx;  // the group's base id is a multiple of 8
  return WideBlock{(int)(off >> 3), (int)((by & ~7u) + (off & 7u))};
}

__host__ __device__ inline int wide_line_regroup(int b, int nb) {
  const int q = nb >> 3;
  if (b >= 8 * q) return b;
  return (b & 7) * q + (b >> 3);
}

}  // namespace ctm
