// Workgroup -> item lookup of the grouped level launches: the items of one
// launch hold ascending first-workgroup indices (blk, the first item's 0,
// also kept in a compact array beside the items), and a workgroup serves the
// last item whose first index it has reached.
#pragma once
#include <hip/hip_runtime.h>

#include <climits>

#include "device.hpp"

namespace qtn {

// Item index of this workgroup; *rank / *count: its position among the
// item's workgroups and their number. One vector load of 64 first indices
// and a ballot per 64 items: no chain of dependent loads (the workgroups of
// a grouped launch are short, so the lookup is a large part of their time).
// All lanes of every wave must be active.
__device__ __forceinline__ int group_item(const int32_t *__restrict__ blk, int n, int *rank, int *count) {
  const int b = (int)blockIdx.x;
  const int lane = (int)(threadIdx.x & 63);
  int idx = 0, end = (int)gridDim.x;
  for (int c0 = 0; c0 < n; c0 += 64) {
    const int i = c0 + lane;
    const int v = i < n ? blk[i] : INT_MAX;
    const int cnt = __popcll(__ballot(v <= b));  // ascending: the items at or before b form a prefix
    if (cnt > 0) idx = c0 + cnt - 1;
    if (cnt < 64) {  // this chunk holds the first item past b, or the list ends in it
      if (c0 + cnt < n) end = __builtin_amdgcn_readlane(v, cnt);
      break;
    }
  }
  const int first = blk[idx];
  *rank = b - first;
  *count = end - first;
  return idx;
}

}  // namespace qtn
