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

// XCD-aware order of the same tiles.  Workgroup ids are dealt to the 8 XCDs
// round robin (id mod 8), and each XCD has its own L2.  Tiles are grouped
// into 8x8 super-tiles (row blocks 8sa..8sa+7, column blocks 8sb..8sb+7),
// the super-tiles ordered longest first; all 64 tiles of super-tile g get
// ids congruent to g mod 8, so they run on one XCD, 32 at a time, and share
// its L2: the tiles running together read the rows of 4 row blocks and 8
// column blocks instead of 32 + 32.  Returns false for the padding ids
// (below the diagonal or past the last block), which do no work.
__device__ __forceinline__ bool tile_xcd_grouped(int64_t id, int64_t nb, int64_t* bi,
                                                 int64_t* bj) {
  const int64_t nbs = (nb + 7) / 8;
  const int64_t x = id & 7, r = id >> 9, t = (id >> 3) & 63;
  const int64_t g = 8 * r + x;
  if (g >= nbs * (nbs + 1) / 2) return false;
  int64_t sa, sb;
  tri_tile_longest_first(g, nbs, &sa, &sb);
  *bi = 8 * sa + (t >> 3);
  *bj = 8 * sb + (t & 7);
  return *bi <= *bj && *bj < nb;
}

// Number of workgroup ids tile_xcd_grouped needs for nb blocks.
__host__ __device__ inline int64_t xcd_grouped_ids(int64_t nb) {
  const int64_t nbs = (nb + 7) / 8;
  const int64_t ns = nbs * (nbs + 1) / 2;
  return (ns + 7) / 8 * 512;
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

// Sum over the 64 lanes as a wave-uniform value, without LDS: DPP row
// shifts by 1, 2, 4, 8 leave each row of 16 lanes with its prefix sums (lane
// 15 of the row holds the row's total), row_bcast:15 adds row 0's total to
// row 1 and row 2's to row 3, row_bcast:31 adds lane 31 (rows 0-1) to rows
// 2-3, and lane 63 ends with the total.  Lanes a shift or broadcast does not
// reach add 0.
__device__ __forceinline__ uint32_t wave_total_u32(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false);  // row_shr:1
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false);  // row_shr:2
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false);  // row_shr:4
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false);  // row_shr:8
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);  // row_bcast:15
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);  // row_bcast:31
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// popcount(x) + c as one v_bcnt_u32_b32, so accumulation stays a chain of
// bcnt ops instead of being regrouped into extra adds.
__device__ __forceinline__ uint32_t bcnt_acc(uint32_t x, uint32_t c) {
  uint32_t r;
  asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(r) : "v"(x), "v"(c));
  return r;
}

// Work item of a persistent workgroup in round k: items are sorted longest
// first and dealt in snake order (round k goes left to right when k is
// even, right to left when odd), so every workgroup gets a similar mix of
// long and short items.  A static schedule: no queue, no atomics, and the
// loop bound is uniform, so every lane leaves the loop in the same
// iteration.
__device__ __forceinline__ int64_t snake_item(int64_t k) {
  const int64_t G = gridDim.x, w = blockIdx.x;
  return k * G + ((k & 1) ? G - 1 - w : w);
}

}  // namespace cs
