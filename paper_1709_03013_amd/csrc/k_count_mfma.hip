// k_count_mfma.hip -- interval counting as an int8 matrix-core contraction.
//
// With U the strictly upper-triangular part of the causal matrix (U[i][k] = 1
// iff i < k and i ~ k), the number of elements inside the interval of a pair
// i < j is m_ij = sum_k U[i][k] U[k][j]: exactly the masked AND + popcount of
// Fig. 2 / Alg. 5, written as an integer matrix product.  Because the stored
// matrix is symmetric, U[k][j] = bit k of row j for k < j, so both operands
// are rows of the packed matrix: row i masked to columns > i ("future of i")
// and row j masked to columns < j ("past of j"), contracted over k.  0/1
// products summed in int32 are exact (m <= N - 2 < 2^31).
//
// gfx950 design: v_mfma_i32_32x32x32_i8.  A workgroup of 8 waves owns a
// 256x256 tile of pairs (row block BI <= column block BJ) and walks the
// 64-bit words 4BI .. 4BJ+3 of its 512 rows (only there can both masks be
// nonzero).  Each of its 8 waves computes 128x64 pairs as 4x2 MFMA tiles.  Per word,
// lane l reads word w of its row (l%32) for each of its 4 A and 4 B
// fragments and keeps the half selected by l/32; the 32 bits D are spread to
// bytes as (D >> r) & 0x01010101, r = 0..7: dwords 0-3 feed the first MFMA,
// 4-7 the second.  A and B use the same spreading, and the hardware uses the
// same k order for A and B, so every bit of the word meets its partner
// exactly once: two MFMAs per word contract all 64 columns.  Masks are only
// applied in the four words of each diagonal block.  The epilogue keeps pairs
// with i < j and bit (i, j) set, bins m, and adds R and the sum of m, with
// one atomic per counter per wave into the tile's row-block stats.
#include <cstdlib>
#include <type_traits>

#include "cs_device.h"
#include "cs_internal.h"

namespace cs {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int kBT = 256;  // pairs per block-tile side (= row block)

// Columns of word w strictly above label i.
__device__ __forceinline__ uint64_t mask_above(int64_t i, int64_t w) {
  const int64_t wi = i >> 6;
  if (w < wi) return 0ull;
  if (w > wi) return ~0ull;
  return ~((2ull << (i & 63)) - 1);
}

// Columns of word w strictly below label j.
__device__ __forceinline__ uint64_t mask_below(int64_t j, int64_t w) {
  const int64_t wj = j >> 6;
  if (w > wj) return 0ull;
  if (w < wj) return ~0ull;
  return (1ull << (j & 63)) - 1;
}

// Bits r0..r0+3 (each with +8, +16, +24) of D as one 16-byte MFMA operand of
// 0/1 bytes: dword q holds bits r0+q, r0+q+8, r0+q+16, r0+q+24.
__device__ __forceinline__ v4i spread4(uint32_t D, int r0) {
  const uint32_t M = 0x01010101u;
  v4i f;
  f[0] = (int)((D >> r0) & M);
  f[1] = (int)((D >> (r0 + 1)) & M);
  f[2] = (int)((D >> (r0 + 2)) & M);
  f[3] = (int)((D >> (r0 + 3)) & M);
  return f;
}

// The 32 bits of D as one FP4 (e2m1) MFMA operand: nibble p of dword r is
// 1.0 (0b0010) when bit 4p + r of D is set, else 0.  Products of 0/1 values
// summed in fp32 are exact integers up to 2^24 > N.  Only the first four
// dwords of the 8-dword operand are read for FP4.
__device__ __forceinline__ v8i spread_fp4(uint32_t D) {
  const uint32_t M = 0x22222222u;
  v8i f;
  f[0] = (int)((D << 1) & M);
  f[1] = (int)(D & M);
  f[2] = (int)((D >> 1) & M);
  f[3] = (int)((D >> 2) & M);
  f[4] = 0;
  f[5] = 0;
  f[6] = 0;
  f[7] = 0;
  return f;
}

// FP4 contraction of one 32x32 tile over 64 k.  Unit scales (E8M0 127) use
// the scaled encoding; scale operands of 0 make the compiler emit the
// unscaled instruction (UNSCALED), whose products are the same.
template <bool UNSCALED>
__device__ __forceinline__ v16f mma_fp4(const v8i& a, const v8i& b, const v16f& c) {
  if constexpr (UNSCALED)
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 4, 4, 0, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 4, 4, 0, 127, 0, 127);
}

// Weighted spreading.  The k order only has to be the same for A and B;
// the value each set bit stands for may differ between them as long as the
// product is one constant.  Class r of D (bits r, r+8, r+16, r+24 for int8;
// bits r, r+4, ... for fp4) keeps the same k slots as above, but A leaves
// most classes where they are (one AND) and B moves them so that every
// product is 64 (int8: 2^r * 2^(6-r); the count is acc >> 6, exact since
// 64(N-2) < 2^31) or 1.0 (fp4: 0.5*2, 1*1, 2*0.5).  Per 32 bits this takes
// 9 (A) + 15 (B) int8 ops instead of 30, and 5 (A) + 7 (B) fp4 ops
// instead of 14.
__device__ __forceinline__ v4i spread4_wa(uint32_t D, int h) {
  const uint32_t M = 0x01010101u;
  v4i f;
  if (h == 0) {
    f[0] = (int)(D & M);
    f[1] = (int)(D & (M << 1));
    f[2] = (int)(D & (M << 2));
    f[3] = (int)(D & (M << 3));
  } else {
    f[0] = (int)(D & (M << 4));
    f[1] = (int)(D & (M << 5));
    f[2] = (int)(D & (M << 6));
    f[3] = (int)((D >> 7) & M);  // class 7 at bit 0 (bit 7 is the sign)
  }
  return f;
}

__device__ __forceinline__ v4i spread4_wb(uint32_t D, int h) {
  const uint32_t M = 0x01010101u;
  v4i f;
  if (h == 0) {
    f[0] = (int)((D << 6) & (M << 6));
    f[1] = (int)((D << 4) & (M << 5));
    f[2] = (int)((D << 2) & (M << 4));
    f[3] = (int)(D & (M << 3));
  } else {
    f[0] = (int)((D >> 2) & (M << 2));
    f[1] = (int)((D >> 4) & (M << 1));
    f[2] = (int)((D >> 6) & M);
    f[3] = (int)((D >> 1) & (M << 6));
  }
  return f;
}

__device__ __forceinline__ v8i spread_fp4_wa(uint32_t D) {
  v8i f;
  f[0] = (int)(D & 0x11111111u);         // 0.5
  f[1] = (int)(D & 0x22222222u);         // 1.0
  f[2] = (int)(D & 0x44444444u);         // 2.0
  f[3] = (int)((D >> 2) & 0x22222222u);  // 1.0
  f[4] = 0;
  f[5] = 0;
  f[6] = 0;
  f[7] = 0;
  return f;
}

__device__ __forceinline__ v8i spread_fp4_wb(uint32_t D) {
  v8i f;
  f[0] = (int)((D << 2) & 0x44444444u);  // 2.0
  f[1] = (int)(D & 0x22222222u);         // 1.0
  f[2] = (int)((D >> 2) & 0x11111111u);  // 0.5
  f[3] = (int)((D >> 2) & 0x22222222u);  // 1.0
  f[4] = 0;
  f[5] = 0;
  f[6] = 0;
  f[7] = 0;
  return f;
}

// Epilogue of one 256x256 tile.  Lane l holds column j = J0 + 32b + l%32
// and rows i = I0 + 32a + 8(v/4) + 4(l/32) + v%4 of tile (a, b); the
// relation bit (i, j) is bit i of row j (all 32 rows of a tile share one word
// of row j).  In a diagonal tile the bits of rows i >= j are cleared first,
// so every test below is a plain bit test.  With FULL, pairs that are not
// counted add to a spare bin kmax+1 so the LDS atomics need no branch.
template <int TM, int TN, int kThreads, bool FULL, int SHIFT, typename Acc>
__device__ __forceinline__ void mfma_epilogue(const Acc (&acc)[TM][TN], const uint64_t* __restrict__ bits,
                                              int64_t N, int64_t W, int64_t BI, int64_t BJ,
                                              int64_t I0, int64_t J0, int kmax,
                                              uint64_t* __restrict__ rb_stats, uint32_t* lds_hist,
                                              const uint64_t (*pre)[TM] = nullptr) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int r32 = lane & 31, g = lane >> 5;
  uint32_t cnt[4] = {0, 0, 0, 0};
  uint32_t nrel = 0;
  // a lane sums at most 16*TM*TN <= 256 interval sizes m <= N - 2; a matrix
  // of 2^21 or more elements needs at least 2^39 bytes, more than a device
  // holds, so the lane's sum fits 32 bits
  uint32_t lsum = 0;
  uint64_t* st = rb_stats + BI * (int64_t)(kmax + 3);
  const uint32_t lb = (uint32_t)(kmax + 1 < kLdsBins ? kmax + 1 : kLdsBins);
#pragma unroll
  for (int b = 0; b < TN; ++b) {
    const int64_t j = J0 + 32 * b + r32;
#pragma unroll
    for (int a = 0; a < TM; ++a) {
      const int64_t ibase = I0 + 32 * a;
      const uint64_t rw = pre ? pre[b][a] : (j < N ? bits[j * W + (ibase >> 6)] : 0ull);
      uint32_t r = (uint32_t)(rw >> (ibase & 63));
      if (BI == BJ) {
        const int64_t lim = j - ibase;  // rows ri < lim have i < j
        r &= lim >= 32 ? ~0u : (lim <= 0 ? 0u : ((1u << lim) - 1u));
      }
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int ri = 8 * (v >> 2) + 4 * g + (v & 3);
        const bool valid = (r >> ri) & 1u;
        const uint32_t m = (uint32_t)acc[a][b][v] >> SHIFT;
        nrel += valid ? 1u : 0u;
        lsum += valid ? m : 0u;
        if constexpr (FULL) {
          // related pairs only: sending the others to a spare bin made half
          // of every tile's LDS atomics hit one address
          if (valid && m < lb) atomicAdd(&lds_hist[m], 1u);
          if (valid && m >= lb && m <= (uint32_t)kmax)
            atomicAdd((unsigned long long*)&st[m], 1ull);
        } else {
#pragma unroll
          for (int k = 0; k < 4; ++k) cnt[k] += (valid && m == (uint32_t)k) ? 1u : 0u;
        }
      }
    }
  }
  nrel = wave_sum_u32(nrel);
  const uint64_t summ = wave_sum_u64(lsum);
  if constexpr (!FULL) {
#pragma unroll
    for (int k = 0; k < 4; ++k) cnt[k] = wave_sum_u32(cnt[k]);
    if (lane < 4) {
      const uint32_t v = lane == 0 ? cnt[0] : lane == 1 ? cnt[1] : lane == 2 ? cnt[2] : cnt[3];
      if (v) atomicAdd((unsigned long long*)&st[lane], (unsigned long long)v);
    }
  } else {
    __syncthreads();
    for (int b = tid; b < (int)lb; b += kThreads) {
      const uint32_t v = lds_hist[b];
      if (v) atomicAdd((unsigned long long*)&st[b], (unsigned long long)v);
    }
  }
  if (lane == 0) {
    if (nrel) atomicAdd((unsigned long long*)&st[kmax + 1], (unsigned long long)nrel);
    if (summ) atomicAdd((unsigned long long*)&st[kmax + 2], (unsigned long long)summ);
  }
}

// One chunk of 4 words (256 columns k) for a wave's TM x TN tiles: xa / xb
// hold the lane's 16 bytes (words 4c + 2g, 4c + 2g + 1) of its row in every A
// and B tile; dword q is half q&1 of word 4c + 2g + q/2.  Masks (first and
// last chunk only), spreading and the MFMAs.
template <int TM, int TN, bool FP4, bool WEIGHTED, bool UNSCALED = false, typename Acc>
__device__ __forceinline__ void mfma_chunk(Acc (&acc)[TM][TN], uint32_t (&xa)[TM][4],
                                           uint32_t (&xb)[TN][4], int64_t I0, int64_t J0,
                                           int64_t c, bool mask_a, bool mask_b) {
  const int lane = threadIdx.x & 63;
  const int r32 = lane & 31, g = lane >> 5;
  if (mask_a) {
#pragma unroll
    for (int t = 0; t < TM; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        xa[t][q] &= (uint32_t)(mask_above(I0 + 32 * t + r32, 4 * c + 2 * g + (q >> 1)) >> (32 * (q & 1)));
  }
  if (mask_b) {
#pragma unroll
    for (int t = 0; t < TN; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        xb[t][q] &= (uint32_t)(mask_below(J0 + 32 * t + r32, 4 * c + 2 * g + (q >> 1)) >> (32 * (q & 1)));
  }
  if constexpr (FP4) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      v8i fa[TM], fb[TN];
#pragma unroll
      for (int t = 0; t < TM; ++t) fa[t] = WEIGHTED ? spread_fp4_wa(xa[t][q]) : spread_fp4(xa[t][q]);
#pragma unroll
      for (int t = 0; t < TN; ++t) fb[t] = WEIGHTED ? spread_fp4_wb(xb[t][q]) : spread_fp4(xb[t][q]);
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b)
          acc[a][b] = mma_fp4<UNSCALED>(fa[a], fb[b], acc[a][b]);
    }
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        v4i fa[TM], fb[TN];
#pragma unroll
        for (int t = 0; t < TM; ++t) fa[t] = WEIGHTED ? spread4_wa(xa[t][q], h) : spread4(xa[t][q], 4 * h);
#pragma unroll
        for (int t = 0; t < TN; ++t) fb[t] = WEIGHTED ? spread4_wb(xb[t][q], h) : spread4(xb[t][q], 4 * h);
#pragma unroll
        for (int a = 0; a < TM; ++a)
#pragma unroll
          for (int b = 0; b < TN; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[a], fb[b], acc[a][b], 0, 0, 0);
      }
  }
}

// The same chunk, software-pipelined: the weighted spreading of step s+1
// (a step = one MFMA per tile pair: a dword q for fp4, a (q, h) half for
// int8) is computed while the MFMAs of step s run, and the scheduler is told
// to interleave them (one MFMA, then a few VALU instructions), so that a
// wave keeps the matrix core busy while its own VALU work proceeds.
template <int TM, int TN, bool FP4, typename Acc>
__device__ __forceinline__ void mfma_chunk_pipelined(Acc (&acc)[TM][TN], uint32_t (&xa)[TM][4],
                                                     uint32_t (&xb)[TN][4], int64_t I0, int64_t J0,
                                                     int64_t c, bool mask_a, bool mask_b) {
  const int lane = threadIdx.x & 63;
  const int r32 = lane & 31, g = lane >> 5;
  if (mask_a) {
#pragma unroll
    for (int t = 0; t < TM; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        xa[t][q] &= (uint32_t)(mask_above(I0 + 32 * t + r32, 4 * c + 2 * g + (q >> 1)) >> (32 * (q & 1)));
  }
  if (mask_b) {
#pragma unroll
    for (int t = 0; t < TN; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        xb[t][q] &= (uint32_t)(mask_below(J0 + 32 * t + r32, 4 * c + 2 * g + (q >> 1)) >> (32 * (q & 1)));
  }
  constexpr int kSteps = FP4 ? 4 : 8;
  constexpr int kValu = FP4 ? 5 : 6;  // VALU instructions placed after each MFMA
  using Op = typename std::conditional<FP4, v8i, v4i>::type;
  Op fa[2][TM], fb[2][TN];
  auto spread = [&](int s, int buf) {
#pragma unroll
    for (int t = 0; t < TM; ++t) {
      if constexpr (FP4) fa[buf][t] = spread_fp4_wa(xa[t][s]);
      else fa[buf][t] = spread4_wa(xa[t][s >> 1], s & 1);
    }
#pragma unroll
    for (int t = 0; t < TN; ++t) {
      if constexpr (FP4) fb[buf][t] = spread_fp4_wb(xb[t][s]);
      else fb[buf][t] = spread4_wb(xb[t][s >> 1], s & 1);
    }
  };
  spread(0, 0);
#pragma unroll
  for (int s = 0; s < kSteps; ++s) {
    const int cur = s & 1;
    if (s + 1 < kSteps) spread(s + 1, cur ^ 1);
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
      for (int b = 0; b < TN; ++b) {
        if constexpr (FP4)
          acc[a][b] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(fa[cur][a], fb[cur][b], acc[a][b],
                                                                     4, 4, 0, 127, 0, 127);
        else
          acc[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[cur][a], fb[cur][b], acc[a][b], 0, 0, 0);
      }
#pragma unroll
    for (int k = 0; k < TM * TN; ++k) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);      // one MFMA
      __builtin_amdgcn_sched_group_barrier(0x002, kValu, 0);  // then VALU work
    }
  }
}

// WM x WN waves over the 256x256 tile; each wave owns (256/WM) x (256/WN)
// pairs as TM x TN tiles of 32x32.  FP4 selects the e2m1 contraction
// (v_mfma_scale_f32_32x32x64_f8f6f4, unit scales) instead of int8: one MFMA
// per 32 bits of each operand row instead of two.
// One 256x256 tile of pairs (row block BI <= column block BJ) by one
// workgroup.  lds_hist (FULL only) holds lb+1 zeroed bins, lb =
// min(kmax+1, kLdsBins) (the last one a spare); larger sizes go straight to
// the row-block stats.
template <int WM, int WN, bool FULL, bool FP4 = false>
__device__ __forceinline__ void mfma_tile(const uint64_t* __restrict__ bits, int64_t N,
                                          int64_t W, int64_t BI, int64_t BJ, int kmax,
                                          uint64_t* __restrict__ rb_stats,
                                          uint32_t* lds_hist) {
  constexpr int kThreads = 64 * WM * WN;
  constexpr int TM = kBT / WM / 32;
  constexpr int TN = kBT / WN / 32;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int r32 = lane & 31, g = lane >> 5;
  const int64_t I0 = BI * kBT + (wave / WN) * (32 * TM);
  const int64_t J0 = BJ * kBT + (wave % WN) * (32 * TN);

  // Words are consumed in chunks of four (32 bytes of every row).  Lane
  // group g reads the 16 bytes holding words 2g and 2g+1 of the chunk for its
  // row l%32 of every A and B tile.  Addresses are a uniform base (the block
  // tile's first row, which always exists) plus a 32-bit per-lane offset;
  // rows past N read that first row instead: their pairs are dropped in the
  // epilogue, so the values never matter.
  const char* abase = (const char*)(bits + BI * kBT * W) + 16 * g;
  const char* bbase = (const char*)(bits + BJ * kBT * W) + 16 * g;
  uint32_t aoffs[TM], boffs[TN];
#pragma unroll
  for (int t = 0; t < TM; ++t) {
    const int64_t rel = I0 - BI * kBT + 32 * t + r32;
    aoffs[t] = BI * kBT + rel < N ? (uint32_t)(rel * W * 8) : 0u;
  }
#pragma unroll
  for (int t = 0; t < TN; ++t) {
    const int64_t rel = J0 - BJ * kBT + 32 * t + r32;
    boffs[t] = BJ * kBT + rel < N ? (uint32_t)(rel * W * 8) : 0u;
  }

  using Acc = typename std::conditional<FP4, v16f, v16i>::type;
  Acc acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[a][b][v] = 0;

  const int64_t c0 = BI, c1 = BJ;  // chunk index = block index (4 words each)
  uint4 na[TM], nbw[TN];
  auto load_chunk = [&](int64_t c) {
    const char* pa = abase + c * 32;
    const char* pb = bbase + c * 32;
#pragma unroll
    for (int t = 0; t < TM; ++t) na[t] = *(const uint4*)(pa + aoffs[t]);
#pragma unroll
    for (int t = 0; t < TN; ++t) nbw[t] = *(const uint4*)(pb + boffs[t]);
  };
  // One chunk: issue the next chunk's loads, mask (diagonal chunks only),
  // spread to int8 and run eight MFMAs per tile pair.  Dword q of a lane's
  // 16 bytes is half q&1 of word 4c + 2g + q/2.
  auto step = [&](int64_t c, bool mask_a, bool mask_b) {
    uint32_t xa[TM][4], xb[TN][4];
#pragma unroll
    for (int t = 0; t < TM; ++t) {
      xa[t][0] = na[t].x; xa[t][1] = na[t].y; xa[t][2] = na[t].z; xa[t][3] = na[t].w;
    }
#pragma unroll
    for (int t = 0; t < TN; ++t) {
      xb[t][0] = nbw[t].x; xb[t][1] = nbw[t].y; xb[t][2] = nbw[t].z; xb[t][3] = nbw[t].w;
    }
    load_chunk(c < c1 ? c + 1 : c1);
    mfma_chunk<TM, TN, FP4, false>(acc, xa, xb, I0, J0, c, mask_a, mask_b);
  };
  load_chunk(c0);
  if (c0 == c1) {
    step(c0, true, true);
  } else {
    step(c0, true, false);
    for (int64_t c = c0 + 1; c < c1; ++c) step(c, false, false);
    step(c1, false, true);
  }

  mfma_epilogue<TM, TN, kThreads, FULL, 0>(acc, bits, N, W, BI, BJ, I0, J0, kmax, rb_stats, lds_hist);
}

// ---- LDS-staged form -------------------------------------------------------
// The chunks of the tile's 512 rows (256 A rows of block BI, 256 B rows of
// block BJ) travel global -> LDS by 16-byte LDS DMA loads (no registers, no
// VALU), S chunks in flight, so the wait for memory overlaps S-1 chunks of
// MFMA work.  A stage is 1024 slots of 16 bytes: slot 2r + s holds half
// s ^ f(r), f(r) = bit 2 of r XOR bit 3 of r, of stage row r (rows 0..255 =
// A, 256..511 = B).  The 16 lanes of rows r..r+15 reading one half then hit
// 16 different 16-byte bank groups (slot mod 16 distinct: rows r and r+8
// differ in f), and so do any 8 of them mod 8 (rows r and r+4 differ in f),
// whether a ds_read_b128 pass serves 8 or 16 lanes; two neighbouring lanes of
// a DMA load read the two halves of one row (32 contiguous bytes).  Each row is read from global memory once
// per workgroup instead of once per wave that uses it.
constexpr int kStageBytes = 512 * 32;

__device__ __forceinline__ int stage_swz(int r) { return ((r >> 2) ^ (r >> 3)) & 1; }

__device__ __forceinline__ uint32_t stage_slot(int r, int half) {
  return (uint32_t)(2 * r + (half ^ stage_swz(r)));
}

template <int WM, int WN, bool FULL, bool FP4, int S, bool WEIGHTED, bool PIPE = false,
          bool UNSCALED = false, bool XPF = false>
__device__ __forceinline__ void mfma_tile_lds(const uint64_t* __restrict__ bits, int64_t N,
                                              int64_t W, int64_t BI, int64_t BJ, int kmax,
                                              uint64_t* __restrict__ rb_stats,
                                              uint32_t* lds_hist, char* stages) {
  constexpr int kWaves = WM * WN;
  constexpr int kThreads = 64 * kWaves;
  constexpr int TM = kBT / WM / 32;
  constexpr int TN = kBT / WN / 32;
  constexpr int L = 1024 / kThreads;  // DMA loads per wave per chunk
  static_assert(L * kThreads == 1024 && S >= 2 && L * (S - 2) <= 63, "bad stage shape");
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int r32 = lane & 31, g = lane >> 5;
  const int64_t I0 = BI * kBT + (wave / WN) * (32 * TM);
  const int64_t J0 = BJ * kBT + (wave % WN) * (32 * TN);

  // DMA load p of this wave fills slots (wave*L + p)*64 + lane of a stage:
  // stage row r = slot/2 (A if r < 256), half from the swizzle.  Global
  // address = uniform block base + 32c + a 32-bit lane offset; rows past N
  // read the block's first row (their pairs are dropped in the epilogue).
  const char* gbase[L];
  uint32_t goff[L];
#pragma unroll
  for (int p = 0; p < L; ++p) {
    const int slot0 = (wave * L + p) * 64;  // uniform
    const bool side_b = slot0 >= 512;
    const int slot = slot0 + lane;
    const int r = (slot >> 1) & 255;
    const int half = (slot & 1) ^ stage_swz(r);
    const int64_t blk = side_b ? BJ : BI;
    gbase[p] = (const char*)(bits + blk * kBT * W);
    const bool valid = blk * kBT + r < N;
    goff[p] = (uint32_t)((valid ? (int64_t)r * W * 8 : 0) + 16 * half);
  }
  typedef __attribute__((address_space(3))) void* lds_ptr;
  typedef __attribute__((address_space(1))) const void* global_ptr;
  auto issue = [&](int64_t c, int st) {
#pragma unroll
    for (int p = 0; p < L; ++p)
      __builtin_amdgcn_global_load_lds((global_ptr)(gbase[p] + c * 32 + goff[p]),
                                       (lds_ptr)(stages + st * kStageBytes + (wave * L + p) * 1024),
                                       16, 0, 0);
  };
  // LDS byte offsets of this lane's 16 bytes in every A and B tile.
  uint32_t aoff[TM], boff[TN];
#pragma unroll
  for (int t = 0; t < TM; ++t)
    aoff[t] = 16u * stage_slot((wave / WN) * (32 * TM) + 32 * t + r32, g);
#pragma unroll
  for (int t = 0; t < TN; ++t)
    boff[t] = 16u * stage_slot(256 + (wave % WN) * (32 * TN) + 32 * t + r32, g);

  using Acc = typename std::conditional<FP4, v16f, v16i>::type;
  Acc acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[a][b][v] = 0;

  const int64_t c0 = BI, c1 = BJ;
  auto read_frags = [&](int stg, uint32_t (&ya)[TM][4], uint32_t (&yb)[TN][4]) {
    const char* sb = stages + stg * kStageBytes;
#pragma unroll
    for (int t = 0; t < TM; ++t) {
      const uint4 v = *(const uint4*)(sb + aoff[t]);
      ya[t][0] = v.x; ya[t][1] = v.y; ya[t][2] = v.z; ya[t][3] = v.w;
    }
#pragma unroll
    for (int t = 0; t < TN; ++t) {
      const uint4 v = *(const uint4*)(sb + boff[t]);
      yb[t][0] = v.x; yb[t][1] = v.y; yb[t][2] = v.z; yb[t][3] = v.w;
    }
  };
  auto chunk = [&](uint32_t (&ya)[TM][4], uint32_t (&yb)[TN][4], int64_t c) {
    if constexpr (PIPE)
      mfma_chunk_pipelined<TM, TN, FP4>(acc, ya, yb, I0, J0, c, c == c0, c == c1);
    else
      mfma_chunk<TM, TN, FP4, WEIGHTED, UNSCALED>(acc, ya, yb, I0, J0, c, c == c0, c == c1);
  };
  if constexpr (XPF) {
    // The epilogue's relation words are loaded first (they arrive during the
    // tile), and each chunk's operands are read from LDS one chunk ahead, so
    // neither latency stalls the matrix core.  S stages hold chunks c..c+S-1
    // at step c; the stage of chunk c is refilled (with chunk c+S) once every
    // wave has read it, which the barrier of step c guarantees.
    uint64_t pre[TN][TM];
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int a = 0; a < TM; ++a) {
        const int64_t j = J0 + 32 * b + r32;
        pre[b][a] = j < N ? bits[j * W + ((I0 + 32 * a) >> 6)] : 0ull;
      }
#pragma unroll
    for (int k = 0; k < S; ++k) issue(c0 + k <= c1 ? c0 + k : c1, k);
    asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)\n\ts_barrier" ::"n"(L * (S - 1)) : "memory");
    uint32_t xa[TM][4], xb[TN][4], na[TM][4], nb[TN][4];
    read_frags(0, xa, xb);
    int st = 0;
    // One step: make chunk c+1 ready, refill chunk c's stage, read chunk
    // c+1 into (ya, yb), contract chunk c from (xa2, xb2).  Two steps per
    // iteration swap the register sets without copies.
    auto step = [&](int64_t c, uint32_t (&cur_a)[TM][4], uint32_t (&cur_b)[TN][4],
                    uint32_t (&nxt_a)[TM][4], uint32_t (&nxt_b)[TN][4]) {
      asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)\n\ts_barrier" ::"n"(L * (S - 2)) : "memory");
      issue(c + S <= c1 ? c + S : c1, st);
      const int nst = st == S - 1 ? 0 : st + 1;
      if (c < c1) read_frags(nst, nxt_a, nxt_b);
      chunk(cur_a, cur_b, c);
      st = nst;
    };
    int64_t c = c0;
    for (; c + 1 <= c1; c += 2) {
      step(c, xa, xb, na, nb);
      step(c + 1, na, nb, xa, xb);
    }
    if (c <= c1) step(c, xa, xb, na, nb);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    mfma_epilogue<TM, TN, kThreads, FULL, ((WEIGHTED || PIPE) && !FP4) ? 6 : 0>(
        acc, bits, N, W, BI, BJ, I0, J0, kmax, rb_stats, lds_hist, pre);
    return;
  }
  // (c0, c1 as above)
  // Prologue: chunks c0 .. c0+S-2 (clamped to c1: a clamped load refills a
  // stage nobody reads again, so every wave always has the same number of
  // loads in flight and the wait count below is a constant).
#pragma unroll
  for (int k = 0; k < S - 1; ++k) issue(c0 + k <= c1 ? c0 + k : c1, k);
  int st = 0;
  for (int64_t c = c0; c <= c1; ++c) {
    // This wave's loads of chunk c are done when at most L*(S-2) (chunks
    // c+1 .. c+S-2) are outstanding; the barrier makes every wave's part of
    // the stage visible and guarantees that every wave finished reading the
    // stage about to be refilled (its LDS reads completed before it came).
    asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)\n\ts_barrier" ::"n"(L * (S - 2)) : "memory");
    const int64_t cn = c + S - 1 <= c1 ? c + S - 1 : c1;
    issue(cn, st == 0 ? S - 1 : st - 1);
    const char* sb = stages + st * kStageBytes;
    uint32_t xa[TM][4], xb[TN][4];
#pragma unroll
    for (int t = 0; t < TM; ++t) {
      const uint4 v = *(const uint4*)(sb + aoff[t]);
      xa[t][0] = v.x; xa[t][1] = v.y; xa[t][2] = v.z; xa[t][3] = v.w;
    }
#pragma unroll
    for (int t = 0; t < TN; ++t) {
      const uint4 v = *(const uint4*)(sb + boff[t]);
      xb[t][0] = v.x; xb[t][1] = v.y; xb[t][2] = v.z; xb[t][3] = v.w;
    }
    if constexpr (PIPE)
      mfma_chunk_pipelined<TM, TN, FP4>(acc, xa, xb, I0, J0, c, c == c0, c == c1);
    else
      mfma_chunk<TM, TN, FP4, WEIGHTED, UNSCALED>(acc, xa, xb, I0, J0, c, c == c0, c == c1);
    st = st == S - 1 ? 0 : st + 1;
  }
  // No LDS DMA may still be writing when the stages are reused or freed.
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");

  mfma_epilogue<TM, TN, kThreads, FULL, ((WEIGHTED || PIPE) && !FP4) ? 6 : 0>(acc, bits, N, W, BI, BJ, I0, J0,
                                                                   kmax, rb_stats, lds_hist);
}

template <int WM, int WN, bool FULL, bool FP4, int S, bool WEIGHTED, bool PIPE, bool GROUPED,
          bool UNSCALED, bool XPF>
__global__ __launch_bounds__(64 * WM * WN, 1) void k_count_mfma_lds(
    const uint64_t* __restrict__ bits, int64_t N, int64_t W, int64_t nb,
    int kmax, uint64_t* __restrict__ rb_stats) {
  extern __shared__ __align__(16) char smem[];  // S stages, then (FULL) lb+1 bins
  uint32_t* lds_hist = (uint32_t*)(smem + S * kStageBytes);
  int64_t BI, BJ;
  if constexpr (GROUPED) {
    if (!tile_xcd_grouped((int64_t)blockIdx.x, nb, &BI, &BJ)) return;  // whole workgroup
  } else {
    tri_tile_longest_first((int64_t)blockIdx.x, nb, &BI, &BJ);
  }
  if constexpr (FULL) {
    const int lb = kmax + 1 < kLdsBins ? kmax + 1 : kLdsBins;
    for (int b = threadIdx.x; b <= lb; b += 64 * WM * WN) lds_hist[b] = 0;
    __syncthreads();
  }
  mfma_tile_lds<WM, WN, FULL, FP4, S, WEIGHTED, PIPE, UNSCALED, XPF>(bits, N, W, BI, BJ, kmax,
                                                                     rb_stats, lds_hist, smem);
}

template <int WM, int WN, bool FULL, bool FP4>
__global__ __launch_bounds__(64 * WM * WN, 1) void k_count_mfma(
    const uint64_t* __restrict__ bits, int64_t N, int64_t W, int64_t nb,
    int kmax, uint64_t* __restrict__ rb_stats) {
  extern __shared__ uint32_t lds_hist[];  // FULL only: lb+1 bins
  int64_t BI, BJ;
  tri_tile_longest_first((int64_t)blockIdx.x, nb, &BI, &BJ);
  if constexpr (FULL) {
    const int lb = kmax + 1 < kLdsBins ? kmax + 1 : kLdsBins;
    for (int b = threadIdx.x; b <= lb; b += 64 * WM * WN) lds_hist[b] = 0;
    __syncthreads();
  }
  mfma_tile<WM, WN, FULL, FP4>(bits, N, W, BI, BJ, kmax, rb_stats, lds_hist);
}

// Batched, persistent: each workgroup takes (set, BI, BJ) items, sorted
// longest first, in snake order until none is left.
template <bool LDS>
__global__ __launch_bounds__(512, 1) void k_batch_count_mfma(BatchDev b) {
  extern __shared__ __align__(16) char smem[];  // LDS form: 4 stages
  for (int64_t k = 0;; ++k) {
    const int64_t it = snake_item(k);
    if (it >= b.n_mfma) break;
    int64_t set, BI, BJ;
    unpack_item(b.mfma_items[it], &set, &BI, &BJ);
    const BatchSet bs = b.sets[set];
    if constexpr (LDS)
      // fp4 (unscaled encoding, weighted spreading): exact for the batch's
      // N <= 16384 < 2^24, and faster than int8
      mfma_tile_lds<2, 4, false, true, 4, true, false, true>(b.bits + bs.bits_off, bs.N, bs.W, BI, BJ, 3,
                                           b.stats + bs.stats_off, nullptr, smem);
    else
      mfma_tile<2, 4, false>(b.bits + bs.bits_off, bs.N, bs.W, BI, BJ, 3, b.stats + bs.stats_off,
                             nullptr);
  }
}

template <int WM, int WN, bool FP4>
hipError_t launch_variant(const uint64_t* bits, int64_t N, int64_t W, int kmax,
                          uint64_t* rb_stats, hipStream_t st) {
  const int64_t nb = (N + kBT - 1) / kBT;
  const int64_t ntiles = nb * (nb + 1) / 2;
  if (ntiles > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 block(64 * WM * WN);
  if (kmax <= 3) {
    hipLaunchKernelGGL((k_count_mfma<WM, WN, false, FP4>), dim3((unsigned)ntiles), block, 0, st,
                       bits, N, W, nb, kmax, rb_stats);
  } else {
    const size_t lds = (size_t)((kmax + 1 < kLdsBins ? kmax + 1 : kLdsBins) + 1) * sizeof(uint32_t);
    hipLaunchKernelGGL((k_count_mfma<WM, WN, true, FP4>), dim3((unsigned)ntiles), block, lds, st,
                       bits, N, W, nb, kmax, rb_stats);
  }
  return hipGetLastError();
}

template <int WM, int WN, bool FP4, int S, bool WEIGHTED = false, bool PIPE = false,
          bool GROUPED = false, bool UNSCALED = false, bool XPF = false>
hipError_t launch_lds_variant(const uint64_t* bits, int64_t N, int64_t W, int kmax,
                              uint64_t* rb_stats, hipStream_t st) {
  const int64_t nb = (N + kBT - 1) / kBT;
  const int64_t ntiles = GROUPED ? xcd_grouped_ids(nb) : nb * (nb + 1) / 2;
  if (ntiles > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 block(64 * WM * WN);
  const size_t stage_bytes = (size_t)S * kStageBytes;
  if (kmax <= 3) {
    hipLaunchKernelGGL((k_count_mfma_lds<WM, WN, false, FP4, S, WEIGHTED, PIPE, GROUPED, UNSCALED, XPF>), dim3((unsigned)ntiles), block,
                       stage_bytes, st, bits, N, W, nb, kmax, rb_stats);
  } else {
    const size_t lds = stage_bytes +
                       (size_t)((kmax + 1 < kLdsBins ? kmax + 1 : kLdsBins) + 1) * sizeof(uint32_t);
    hipLaunchKernelGGL((k_count_mfma_lds<WM, WN, true, FP4, S, WEIGHTED, PIPE, GROUPED, UNSCALED, XPF>), dim3((unsigned)ntiles), block, lds,
                       st, bits, N, W, nb, kmax, rb_stats);
  }
  return hipGetLastError();
}

template <bool FP4>
hipError_t launch_by_variant(int v, const uint64_t* bits, int64_t N, int64_t W, int kmax,
                             uint64_t* rb_stats, hipStream_t st) {
  switch (v) {
    case 0: return launch_variant<2, 2, FP4>(bits, N, W, kmax, rb_stats, st);
    case 1: return launch_variant<2, 4, FP4>(bits, N, W, kmax, rb_stats, st);
    case 2: return launch_lds_variant<2, 4, FP4, 4>(bits, N, W, kmax, rb_stats, st);
    case 3: return launch_lds_variant<2, 2, FP4, 4>(bits, N, W, kmax, rb_stats, st);
    case 4: return launch_lds_variant<2, 4, FP4, 3>(bits, N, W, kmax, rb_stats, st);
    case 5: return launch_lds_variant<2, 2, FP4, 3>(bits, N, W, kmax, rb_stats, st);
    case 6: return launch_lds_variant<2, 4, FP4, 4, true>(bits, N, W, kmax, rb_stats, st);
    case 7: return launch_lds_variant<2, 2, FP4, 3, true>(bits, N, W, kmax, rb_stats, st);
    case 8: return launch_lds_variant<2, 4, FP4, 4, true, true>(bits, N, W, kmax, rb_stats, st);
    case 9: return launch_lds_variant<2, 2, FP4, 3, true, true>(bits, N, W, kmax, rb_stats, st);
    case 10: return launch_lds_variant<2, 4, FP4, 4, true, false, true>(bits, N, W, kmax, rb_stats, st);
    case 11: return launch_lds_variant<2, 4, FP4, 4, true, true, true>(bits, N, W, kmax, rb_stats, st);
    case 12: return launch_lds_variant<2, 4, FP4, 4, true, false, true, true>(bits, N, W, kmax, rb_stats, st);
    default: return launch_lds_variant<2, 4, FP4, 4, true, false, true, true, true>(bits, N, W, kmax, rb_stats, st);
  }
}

}  // namespace

// Kernel shape: 0 = 2x2 waves of 128x128 pairs, 1 = 2x4 waves of 128x64
// pairs (both loading operands straight to registers, one chunk ahead);
// 2..5 = the LDS-staged form with 2x4 / 2x2 waves and 4 / 3 stages; 6, 7 =
// 2x4 waves, 4 stages / 2x2 waves, 3 stages with the weighted spreading; 8,
// 9 = the same, software-pipelined with interleaved MFMA and VALU; 10, 11 =
// 6 and 8 with the XCD-grouped tile order; 12 = 10 with the unscaled fp4
// MFMA encoding; 13 = 12 reading each chunk's operands from LDS one chunk
// ahead and the epilogue's relation words at the start of the tile (no
// faster: LDS latency is not what limits the kernel).
// The default, 12, was
// the fastest on MI355X for both operand types (2D N=2^17: int8 186 ms, fp4
// 110-112 ms; the first LDS-staged form, 2, took 209 / 136 ms and the
// register-staged form, 1, 221 / 176 ms).  The environment variable
// CS_MFMA_VARIANT overrides it for timing.
static int mfma_variant() {
  const char* e = getenv("CS_MFMA_VARIANT");
  return e ? atoi(e) : 12;
}

hipError_t launch_count_mfma(const uint64_t* bits, int64_t N, int64_t W, int kmax,
                             uint64_t* rb_stats, hipStream_t st) {
  static_assert(kBT == kRowBlock, "block tile must equal the stats row block");
  if (N <= 1) return hipSuccess;
  return launch_by_variant<false>(mfma_variant(), bits, N, W, kmax, rb_stats, st);
}

hipError_t launch_count_mfma_fp4(const uint64_t* bits, int64_t N, int64_t W, int kmax,
                                 uint64_t* rb_stats, hipStream_t st) {
  if (N <= 1) return hipSuccess;
  return launch_by_variant<true>(mfma_variant(), bits, N, W, kmax, rb_stats, st);
}

namespace {
template <int WM, int WN, bool FP4, int S, bool WEIGHTED = false, bool PIPE = false,
          bool GROUPED = false, bool UNSCALED = false, bool XPF = false>
hipError_t set_lds_limits() {
  const int stages = S * kStageBytes;
  const int full = stages + (kLdsBins + 1) * (int)sizeof(uint32_t);
  hipError_t e = hipFuncSetAttribute(
      (const void*)k_count_mfma_lds<WM, WN, false, FP4, S, WEIGHTED, PIPE, GROUPED, UNSCALED, XPF>,
      hipFuncAttributeMaxDynamicSharedMemorySize, stages);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(
        (const void*)k_count_mfma_lds<WM, WN, true, FP4, S, WEIGHTED, PIPE, GROUPED, UNSCALED, XPF>,
        hipFuncAttributeMaxDynamicSharedMemorySize, full);
  return e;
}
}  // namespace

// Dynamic LDS limits of the LDS-staged kernels (above the 64 KiB default).
hipError_t init_count_mfma() {
  hipError_t e = hipFuncSetAttribute((const void*)k_batch_count_mfma<true>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, 4 * kStageBytes);
  if (e == hipSuccess) e = set_lds_limits<2, 4, false, 4>();
  if (e == hipSuccess) e = set_lds_limits<2, 2, false, 4>();
  if (e == hipSuccess) e = set_lds_limits<2, 4, false, 3>();
  if (e == hipSuccess) e = set_lds_limits<2, 2, false, 3>();
  if (e == hipSuccess) e = set_lds_limits<2, 4, true, 4>();
  if (e == hipSuccess) e = set_lds_limits<2, 2, true, 4>();
  if (e == hipSuccess) e = set_lds_limits<2, 4, true, 3>();
  if (e == hipSuccess) e = set_lds_limits<2, 2, true, 3>();
  if (e == hipSuccess) e = set_lds_limits<2, 4, false, 4, true>();
  if (e == hipSuccess) e = set_lds_limits<2, 2, false, 3, true>();
  if (e == hipSuccess) e = set_lds_limits<2, 4, true, 4, true>();
  if (e == hipSuccess) e = set_lds_limits<2, 2, true, 3, true>();
  if (e == hipSuccess) e = set_lds_limits<2, 4, false, 4, true, true>();
  if (e == hipSuccess) e = set_lds_limits<2, 2, false, 3, true, true>();
  if (e == hipSuccess) e = set_lds_limits<2, 4, true, 4, true, true>();
  if (e == hipSuccess) e = set_lds_limits<2, 2, true, 3, true, true>();
  if (e == hipSuccess) e = set_lds_limits<2, 4, false, 4, true, false, true>();
  if (e == hipSuccess) e = set_lds_limits<2, 4, true, 4, true, false, true>();
  if (e == hipSuccess) e = set_lds_limits<2, 4, false, 4, true, true, true>();
  if (e == hipSuccess) e = set_lds_limits<2, 4, true, 4, true, true, true>();
  if (e == hipSuccess) e = set_lds_limits<2, 4, false, 4, true, false, true, true>();
  if (e == hipSuccess) e = set_lds_limits<2, 4, true, 4, true, false, true, true>();
  if (e == hipSuccess) e = set_lds_limits<2, 4, false, 4, true, false, true, true, true>();
  if (e == hipSuccess) e = set_lds_limits<2, 4, true, 4, true, false, true, true, true>();
  return e;
}

hipError_t launch_batch_count_mfma(const BatchDev& b, int grid, hipStream_t st) {
  if (b.n_mfma <= 0) return hipSuccess;
  if (mfma_variant() >= 2) {
    const size_t lds = 4 * (size_t)kStageBytes;
    hipLaunchKernelGGL(k_batch_count_mfma<true>, dim3((unsigned)grid), dim3(512), lds, st, b);
  } else {
    hipLaunchKernelGGL(k_batch_count_mfma<false>, dim3((unsigned)grid), dim3(512), 0, st, b);
  }
  return hipGetLastError();
}

}  // namespace cs
