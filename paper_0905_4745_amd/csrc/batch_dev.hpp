// Device-side lookup of a batched launch: which system a workgroup belongs
// to and its block coordinates within that system's own grid.
#pragma once

#include "common.hpp"
#include "kernels.hpp"

namespace mn {

// the system owning workgroup b: the last i with start[i] <= b
__device__ inline int bgrid_find(const BGrid* __restrict__ g, int nsys, int b) {
  int lo = 0, hi = nsys;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (g[mid].start <= b) lo = mid;
    else hi = mid;
  }
  return lo;
}
__device__ inline Bk bgrid_local(const BGrid& g, int local) {
  Bk k;
  k.gx = g.gx;
  k.gy = g.gy;
  k.gz = g.gz;
  k.x = local % g.gx;
  const int r = local / g.gx;
  k.y = r % g.gy;
  k.z = r / g.gy;
  return k;
}

}  // namespace mn
