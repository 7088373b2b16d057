// Order-preserving compaction of support slots by one 1024-thread workgroup (the device
// function of k_compact, also run at the start of the mesh kernel): non-marker slots (and,
// when occ is non-null, those whose pixel is not yet occupied; kept pixels are then marked)
// move to the front in order; the count goes to n_out and, when non-null, to header.
// Chunks of 1024 slots are read completely before any is written.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace sm {

__device__ __forceinline__ void compact_block(sm_support* slots, int n, int* n_out, uint8_t* occ, int W,
                                              int* header) {
  __shared__ int wsum[16];
  __shared__ int wofs[16];
  __shared__ int total;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int base = 0;
  for (int start = 0; start < n; start += 1024) {
    const int i = start + threadIdx.x;
    sm_support s;
    bool keep = false;
    if (i < n) {
      s = slots[i];
      keep = s.d != kPending && s.d != kRejected;
      if (keep && occ) keep = occ[(size_t)s.v * W + s.u] == 0;
    }
    const unsigned long long m = __ballot(keep);
    const int pre = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[w] = __popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
      int acc = 0;
      for (int k = 0; k < 16; ++k) {
        wofs[k] = acc;
        acc += wsum[k];
      }
      total = acc;
    }
    __syncthreads();
    if (keep) {
      slots[base + wofs[w] + pre] = s;
      if (occ) occ[(size_t)s.v * W + s.u] = 1;
    }
    base += total;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *n_out = base;
    if (header) *header = base;
  }
}

}  // namespace sm
