// cs_device.h -- device helpers shared by the counting kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cs {

// Upper-triangular tiles (bi <= bj) of an nb x nb block grid, longest first:
// group q (1..nb) holds the q tiles with bj - bi = nb - q and starts at
// linear index q(q-1)/2.
__device__ __forceinline__ void tri_tile_longest_first(int64_t t, int64_t nb,
                                                       int64_t* bi, int64_t* bj) {
  int64_t q = (int64_t)((__builtin_sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5) + 1;
  while (q > 1 && (q - 1) * q / 2 > t) --q;
  while (q * (q + 1) / 2 <= t) ++q;
  const int64_t off = t - (q - 1) * q / 2;
  *bi = off;
  *bj = off + (nb - q);
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// popcount(x) + c as one v_bcnt_u32_b32, so accumulation stays a chain of
// bcnt ops instead of being regrouped into extra adds.
__device__ __forceinline__ uint32_t bcnt_acc(uint32_t x, uint32_t c) {
  uint32_t r;
  asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(r) : "v"(x), "v"(c));
  return r;
}

// Next work item of a persistent workgroup's queue, the same value in every
// lane.  Every lane issues the atomic but only lane 0 adds 1, so lane 0 gets
// the head before its own increment whatever order the lanes are applied in;
// there is no lane-dependent branch, so the compiler cannot let lanes leave
// a persistent loop in different iterations.  (Kernels using this are built
// with the atomic combiner off, which would reintroduce such a branch.)
__device__ __forceinline__ uint32_t next_item(uint32_t* head) {
  const uint32_t v = atomicAdd(head, threadIdx.x == 0 ? 1u : 0u);
  return __builtin_amdgcn_readlane(v, 0);
}

}  // namespace cs
