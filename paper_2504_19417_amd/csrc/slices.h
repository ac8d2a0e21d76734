// Device-side lookup of the slice that owns an event or a brick (slices lie
// back to back; binary search over their first event / first brick).
#pragma once

#include <hip/hip_runtime.h>

#include "veckm_internal.h"

namespace veckm {

__device__ inline SliceDesc slice_by_event(Batch b, int i) {  // by value: no private copy
  if (b.nslices == 1) return b.s0;
  int lo = 0, hi = b.nslices - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (b.table[mid].ev_off <= i) lo = mid; else hi = mid - 1;
  }
  return b.table[lo];
}

__device__ inline SliceDesc slice_by_brick(Batch b, int gb) {
  if (b.nslices == 1) return b.s0;
  int lo = 0, hi = b.nslices - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (b.table[mid].brick_off <= gb) lo = mid; else hi = mid - 1;
  }
  return b.table[lo];
}

}  // namespace veckm
