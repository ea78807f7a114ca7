// Workgroup -> item lookup of the grouped level launches: the items of one
// launch hold ascending first-workgroup indices (blk0, the first item's 0),
// and a workgroup serves the last item whose blk0 it has reached.
#pragma once
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace qtn {

// Item index of this workgroup; *rank / *count: its position among the
// item's workgroups and their number.
__device__ __forceinline__ int group_item(const LItem *__restrict__ items, int n, int *rank, int *count) {
  int lo = 0, hi = n - 1;
  const int b = (int)blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].blk0 <= b) lo = mid;
    else hi = mid - 1;
  }
  const int end = lo + 1 < n ? items[lo + 1].blk0 : (int)gridDim.x;
  *rank = b - items[lo].blk0;
  *count = end - items[lo].blk0;
  return lo;
}

}  // namespace qtn
