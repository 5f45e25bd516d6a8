// k_count_mfma.hip -- interval counting as a matrix-core contraction.
//
// With U the strictly upper-triangular part of the causal matrix (U[i][k] = 1
// iff i < k and i ~ k), the number of elements inside the interval of a pair
// i < j is m_ij = sum_k U[i][k] U[k][j]: exactly the masked AND + popcount of
// Fig. 2 / Alg. 5, written as an integer matrix product.  Because the stored
// matrix is symmetric, U[k][j] = bit k of row j for k < j, so both operands
// are rows of the packed matrix: row i masked to columns > i ("future of i")
// and row j masked to columns < j ("past of j"), contracted over k.
//
// Two operand types, one kernel shape:
//  * fp4 (e2m1) operands with fp32 accumulation,
//    v_mfma_scale_f32_32x32x64_f8f6f4 with unit scales: products of the
//    values below are exactly 1, so the fp32 sums are exact integers while
//    m < 2^24 (the library refuses N >= 2^24 on this path);
//  * int8 operands with int32 accumulation, v_mfma_i32_32x32x32_i8: every
//    product is 64, exact while 64 (N - 2) < 2^31.
//
// gfx950 design.  A workgroup of 8 waves (2 x 4) owns a 256x256 tile of
// pairs (row block BI <= column block BJ) and walks the 64-bit words
// 4BI .. 4BJ+3 of its 512 rows, where both masks can be nonzero, in chunks
// of four words.  Chunks move global -> LDS by 16-byte LDS-DMA loads
// (no registers, no VALU), four stages in flight; each wave contracts
// 128x64 pairs as 4x2 MFMA tiles of 32x32.  Lane l reads the 16 bytes of
// its row l%32 that hold words 2(l/32) and 2(l/32)+1 of the chunk, and the
// bits are spread to MFMA operands in registers with the weighted spreading
// below.  The hardware uses the same k order for A and B, so every column
// meets its partner exactly once.  Masks are only applied in the first and
// last chunk.  Tiles are dealt XCD-aware (cs_device.h) on large matrices,
// longest first on smaller ones.  The epilogue keeps
// pairs with i < j and bit (i, j) set, bins m, and adds R and the sum of m
// with one atomic per counter per wave into the tile's row-block stats.
#include <type_traits>

#include "cs_device.h"
#include "cs_internal.h"

namespace cs {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef float v16f __attribute__((ext_vector_type(16)));

// Tile shapes: BT x BT pairs per workgroup of WM x WN waves, each wave
// TM x TN MFMA tiles of 32x32 pairs.  The single-set count uses Big; the
// batched count uses Big or Small per set (chosen by the batch tuner).
template <int BT_, int WM_, int WN_>
struct Shape {
  static constexpr int BT = BT_, WM = WM_, WN = WN_;
  static constexpr int Threads = 64 * WM * WN;
  static constexpr int TM = BT / WM / 32, TN = BT / WN / 32;
  static constexpr int StageBytes = 2 * BT * 32;  // a chunk (32 bytes) of BT A and BT B rows
  static constexpr int L = 4 * BT / Threads;      // 16-byte DMA loads per lane per chunk
};
using Big = Shape<256, 2, 4>;
using Small = Shape<128, 2, 2>;
constexpr int kStages = 4;

// Of the 32 columns cb .. cb+31, those at or above cb + s: the shift count
// clamped to 0..32 and one 64-bit shift, so that s >= 32 empties the word.
// Columns above label i: s = i + 1 - cb; below label j: the complement with
// s = j - cb.
__device__ __forceinline__ uint32_t cols_from(int s) {
  const int c = s < 0 ? 0 : (s > 32 ? 32 : s);
  return (uint32_t)(0xFFFFFFFFull << c);
}

// Weighted spreading.  The k order only has to be the same for A and B; the
// value each set bit stands for may differ between them as long as every
// product is one constant.  Bit class r of a 32-bit word D (bits r, r+8,
// r+16, r+24 for int8; bits r, r+4, ... for fp4) occupies the same k slots
// in A and B, but A leaves most classes where they are (one AND) and B moves
// them so that every product is 64 (int8: 2^r * 2^(6-r); the count is
// acc >> 6) or 1.0 (fp4: 0.5*2, 1*1, 2*0.5).  Per 32 bits this takes 9 (A)
// + 15 (B) int8 ops, 5 (A) + 7 (B) fp4 ops.
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

// fp4: nibble p of dword q of the operand covers bit 4p + q of D (only the
// first four dwords of the 8-dword operand are read for fp4).
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

// Interval size m of accumulator element v (fp4: the exact fp32 integer;
// int8: the int32 sum over products of 64).
__device__ __forceinline__ uint32_t acc_count(float x) { return (uint32_t)x; }
__device__ __forceinline__ uint32_t acc_count(int x) { return (uint32_t)x >> 6; }

// a * b + c for a, b < 2^24, and (a << s) + c, each as one instruction.
__device__ __forceinline__ uint32_t mad_u24(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t r;
  asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}
__device__ __forceinline__ uint32_t lshl_add(uint32_t a, uint32_t s, uint32_t c) {
  uint32_t r;
  asm("v_lshl_add_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(s), "v"(c));
  return r;
}

// Epilogue of one 256x256 tile.  Lane l holds column j = J0 + 32b + l%32
// and rows i = I0 + 32a + 8(v/4) + 4(l/32) + v%4 of tile (a, b); the
// relation bit (i, j) is bit i of row j (all 32 rows of a tile share one word
// of row j).  In a diagonal tile the bits of rows i >= j are cleared first,
// so every test below is a plain bit test.  FULL bins every size m <= kmax:
// sizes below kLdsBins in the workgroup's LDS bins (lds_hist, zeroed), larger
// ones straight into the row-block stats.  rel: where the caller kept, in
// LDS, the 16 bytes each lane read of its B rows in the tile's first chunk
// (16 bytes per lane and B tile; the word of rows I0 + 32a is word
// wl0 + a/2 of that chunk), else the relation words are read from memory.
// Its loop over the 16 elements of
// a 32x32 tile is not unrolled: one element's temporaries at a time keep the
// kernel within its registers.
template <class Sh, bool FULL, typename Acc>
__device__ __forceinline__ void mfma_epilogue(const Acc (&acc)[Sh::TM][Sh::TN],
                                              const uint64_t* __restrict__ bits, int64_t N,
                                              int64_t W, int64_t BI, int64_t BJ, int64_t I0,
                                              int64_t J0, int kmax,
                                              uint64_t* __restrict__ rb_stats, uint32_t* lds_hist,
                                              const char* rel = nullptr, int wl0 = 0) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int r32 = lane & 31, g = lane >> 5;
  uint32_t cnt[4] = {0, 0, 0, 0};
  uint32_t pk[2] = {0, 0};
  uint32_t nrel = 0;
  // a lane sums at most 16*TM*TN <= 128 interval sizes m <= N - 2; a matrix
  // of 2^21 or more elements needs at least 2^39 bytes, more than a device
  // holds, so the lane's sum fits 32 bits
  uint32_t lsum = 0;
  uint64_t* st = rb_stats + (BI * Sh::BT / kRowBlock) * (int64_t)(kmax + 3);
  const uint32_t lb = (uint32_t)(kmax + 1 < kLdsBins ? kmax + 1 : kLdsBins);
#pragma unroll
  for (int b = 0; b < Sh::TN; ++b) {
    const int64_t j = J0 + 32 * b + r32;
#pragma unroll
    for (int a = 0; a < Sh::TM; ++a) {
      const int64_t ibase = I0 + 32 * a;
      uint64_t rw = 0ull;
      if (j < N) {
        if (rel) {
          // word wl of the tile's first chunk, kept by the lanes with g = wl / 2
          const int wl = wl0 + (a >> 1);
          rw = *(const uint64_t*)(rel + (b * 64 + r32 + 32 * (wl >> 1)) * 16 + 8 * (wl & 1));
        } else {
          rw = bits[j * W + (ibase >> 6)];
        }
      }
      uint32_t r = (uint32_t)(rw >> (ibase & 63));
      if (BI == BJ) {
        const int64_t lim = j - ibase;  // rows ri < lim have i < j
        r &= lim >= 32 ? ~0u : (lim <= 0 ? 0u : ((1u << lim) - 1u));
      }
      if constexpr (FULL) {
#pragma unroll 1
        for (int v = 0; v < 16; ++v) {
          const int ri = 8 * (v >> 2) + 4 * g + (v & 3);
          const bool valid = (r >> ri) & 1u;
          const uint32_t m = acc_count(acc[a][b][v]);
          nrel += valid ? 1u : 0u;
          lsum += valid ? m : 0u;
          // related pairs only: sending the others to a spare bin made half
          // of every tile's LDS atomics hit one address
          if (valid) {
            if (m < lb)
              atomicAdd(&lds_hist[m], 1u);
            else if (m <= (uint32_t)kmax)
              atomicAdd((unsigned long long*)&st[m], 1ull);
          }
        }
      } else {
        // R: one bit count of the lane's 16 relation bits of the tile.
        // N_0..N_3: 7-bit fields of pk (bits 0, 7, 14, 21; sizes >= 4 go to
        // bits 28.. and their carries leave the word), each half of the
        // lane's tiles (<= 64 pairs) in its own word, so no field overflows.
        nrel = bcnt_acc(r & (0x0F0F0F0Fu << (4 * g)), nrel);
        const int h = (b * Sh::TM + a) < (Sh::TM * Sh::TN) / 2 ? 0 : 1;
        const uint32_t rg = r >> (4 * g);  // element v's bit at 8(v/4) + v%4
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const uint32_t valid = (rg >> (8 * (v >> 2) + (v & 3))) & 1u;
          const uint32_t m = acc_count(acc[a][b][v]);
          if constexpr (std::is_same<Acc, v16f>::value)
            lsum = mad_u24(valid, m, lsum);  // fp4 path: m < 2^24
          else
            lsum += valid ? m : 0u;
          const uint32_t sz = m < 4u ? m : 4u;
          pk[h] = lshl_add(valid, 7u * sz, pk[h]);
        }
      }
    }
  }
  // wave totals (uniform): the sum of m in two 16-bit halves, N_0..N_3 two
  // to a word (at most 128 pairs per lane, 8192 per wave, in 16 bits)
  nrel = wave_total_u32(nrel);
  const uint64_t summ =
      (uint64_t)wave_total_u32(lsum & 0xFFFFu) + ((uint64_t)wave_total_u32(lsum >> 16) << 16);
  if constexpr (!FULL) {
    uint32_t f[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) f[k] = ((pk[0] >> (7 * k)) & 127u) + ((pk[1] >> (7 * k)) & 127u);
    const uint32_t t01 = wave_total_u32(f[0] | (f[1] << 16)), t23 = wave_total_u32(f[2] | (f[3] << 16));
    cnt[0] = t01 & 0xFFFFu;
    cnt[1] = t01 >> 16;
    cnt[2] = t23 & 0xFFFFu;
    cnt[3] = t23 >> 16;
    if (lane < 4) {
      const uint32_t v = lane == 0 ? cnt[0] : lane == 1 ? cnt[1] : lane == 2 ? cnt[2] : cnt[3];
      if (v) atomicAdd((unsigned long long*)&st[lane], (unsigned long long)v);
    }
  } else {
    __syncthreads();
    for (int b = tid; b < (int)lb; b += Sh::Threads) {
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
// last chunk only), weighted spreading and the MFMAs.  Scale operands of 0
// select the unscaled fp4 instruction; its products are the same as with
// unit scales.
template <class Sh, bool FP4, typename Acc>
__device__ __forceinline__ void mfma_chunk(Acc (&acc)[Sh::TM][Sh::TN], uint32_t (&xa)[Sh::TM][4],
                                           uint32_t (&xb)[Sh::TN][4], int64_t I0, int64_t J0,
                                           int64_t c, bool mask_a, bool mask_b) {
  constexpr int kTM = Sh::TM, kTN = Sh::TN;
  const int lane = threadIdx.x & 63;
  const int r32 = lane & 31, g = lane >> 5;
  // dword q of the lane's 16 bytes holds columns cb + 32q .. cb + 32q + 31
  // (a matrix that fits a device has fewer than 2^21 labels, so the
  // differences fit an int)
  const int cb = (int)(256 * c) + 128 * g;
  if (mask_a) {
#pragma unroll
    for (int t = 0; t < kTM; ++t) {
      const int s0 = (int)I0 + 32 * t + r32 + 1 - cb;  // columns above row i
#pragma unroll
      for (int q = 0; q < 4; ++q) xa[t][q] &= cols_from(s0 - 32 * q);
    }
  }
  if (mask_b) {
#pragma unroll
    for (int t = 0; t < kTN; ++t) {
      const int s0 = (int)J0 + 32 * t + r32 - cb;  // columns below row j
#pragma unroll
      for (int q = 0; q < 4; ++q) xb[t][q] &= ~cols_from(s0 - 32 * q);
    }
  }
  if constexpr (FP4) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      v8i fa[kTM], fb[kTN];
#pragma unroll
      for (int t = 0; t < kTM; ++t) fa[t] = spread_fp4_wa(xa[t][q]);
#pragma unroll
      for (int t = 0; t < kTN; ++t) fb[t] = spread_fp4_wb(xb[t][q]);
#pragma unroll
      for (int a = 0; a < kTM; ++a)
#pragma unroll
        for (int b = 0; b < kTN; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(fa[a], fb[b], acc[a][b], 4, 4,
                                                                     0, 0, 0, 0);
    }
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        v4i fa[kTM], fb[kTN];
#pragma unroll
        for (int t = 0; t < kTM; ++t) fa[t] = spread4_wa(xa[t][q], h);
#pragma unroll
        for (int t = 0; t < kTN; ++t) fb[t] = spread4_wb(xb[t][q], h);
#pragma unroll
        for (int a = 0; a < kTM; ++a)
#pragma unroll
          for (int b = 0; b < kTN; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[a], fb[b], acc[a][b], 0, 0, 0);
      }
  }
}

// ---- LDS staging -------------------------------------------------------------
// The chunks of the tile's 2 BT rows (BT A rows of block BI, BT B rows of
// block BJ) travel global -> LDS by 16-byte LDS-DMA loads, kStages chunks in
// flight, so the wait for memory overlaps kStages-1 chunks of MFMA work.  A
// stage is 4 BT slots of 16 bytes: slot 2r + s holds half s ^ f(r),
// f(r) = bit 2 of r XOR bit 3 of r, of stage row r (rows 0..BT-1 = A,
// BT..2BT-1 = B).  The 16 lanes of rows r..r+15 reading one half then hit 16
// different 16-byte bank groups (slot mod 16 distinct: rows r and r+8 differ
// in f), and so do any 8 of them mod 8 (rows r and r+4 differ in f), whether
// a ds_read_b128 pass serves 8 or 16 lanes; two neighbouring lanes of a DMA
// load read the two halves of one row (32 contiguous bytes).  Each row is
// read from global memory once per workgroup instead of once per wave.
__device__ __forceinline__ int stage_swz(int r) { return ((r >> 2) ^ (r >> 3)) & 1; }

__device__ __forceinline__ uint32_t stage_slot(int r, int half) {
  return (uint32_t)(2 * r + (half ^ stage_swz(r)));
}

// One BT x BT tile of pairs (row block BI <= column block BJ, in units of
// BT labels) by one workgroup.  The tile's columns k lie in the 4-word
// chunks BI*BT/256 .. (BJ*BT + BT - 1)/256; the first holds every column at
// or below a row of block BI and the last every column at or above a row of
// block BJ, so masks are applied in those two chunks only.  lds_hist (FULL
// only): min(kmax+1, kLdsBins) zeroed bins.
//
// The waits are hand-counted: before chunk c is read, at most
// L*(kStages-2) of this wave's vector-memory operations may be outstanding
// (the DMA loads of chunks c+1 .. c+kStages-2).  Loads complete in issue
// order, so any other vector-memory operation the compiler adds can only
// make the wait longer, never end it before chunk c has arrived.
template <class Sh, bool FULL, bool FP4>
__device__ __forceinline__ void mfma_tile_lds(const uint64_t* __restrict__ bits, int64_t N,
                                              int64_t W, int64_t BI, int64_t BJ, int kmax,
                                              uint64_t* __restrict__ rb_stats,
                                              uint32_t* lds_hist, char* stages) {
  constexpr int S = kStages;
  constexpr int BT = Sh::BT, TM = Sh::TM, TN = Sh::TN, WN = Sh::WN, L = Sh::L;
  static_assert(L * Sh::Threads == 4 * BT && S >= 2 && L * (S - 2) <= 63, "bad stage shape");
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int r32 = lane & 31, g = lane >> 5;
  const int64_t I0 = BI * BT + (wave / WN) * (32 * TM);
  const int64_t J0 = BJ * BT + (wave % WN) * (32 * TN);

  // DMA load p of this wave fills slots (wave*L + p)*64 + lane of a stage:
  // stage row slot/2 (A below BT), half from the swizzle.  Global address =
  // uniform block base + 32c + a 32-bit lane offset; rows past N read the
  // block's first row (their pairs are dropped in the epilogue).
  const char* gbase[L];
  uint32_t goff[L];
#pragma unroll
  for (int p = 0; p < L; ++p) {
    const int slot0 = (wave * L + p) * 64;  // uniform
    const bool side_b = slot0 >= 2 * BT;
    const int slot = slot0 + lane;
    const int r = (slot >> 1) & (BT - 1);
    const int half = (slot & 1) ^ stage_swz(r);
    const int64_t blk = side_b ? BJ : BI;
    gbase[p] = (const char*)(bits + blk * BT * W);
    const bool valid = blk * BT + r < N;
    goff[p] = (uint32_t)((valid ? (int64_t)r * W * 8 : 0) + 16 * half);
  }
  typedef __attribute__((address_space(3))) void* lds_ptr;
  typedef __attribute__((address_space(1))) const void* global_ptr;
  auto issue = [&](int64_t c, int st) {
#pragma unroll
    for (int p = 0; p < L; ++p)
      __builtin_amdgcn_global_load_lds((global_ptr)(gbase[p] + c * 32 + goff[p]),
                                       (lds_ptr)(stages + st * Sh::StageBytes + (wave * L + p) * 1024),
                                       16, 0, 0);
  };
  // LDS byte offsets of this lane's 16 bytes in every A and B tile.
  uint32_t aoff[TM], boff[TN];
#pragma unroll
  for (int t = 0; t < TM; ++t)
    aoff[t] = 16u * stage_slot((wave / WN) * (32 * TM) + 32 * t + r32, g);
#pragma unroll
  for (int t = 0; t < TN; ++t)
    boff[t] = 16u * stage_slot(BT + (wave % WN) * (32 * TN) + 32 * t + r32, g);

  using Acc = typename std::conditional<FP4, v16f, v16i>::type;
  Acc acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[a][b][v] = 0;

  const int64_t c0 = BI * BT / 256, c1 = (BJ * BT + BT - 1) / 256;  // 4-word chunks
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
    const char* sb = stages + st * Sh::StageBytes;
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
    mfma_chunk<Sh, FP4>(acc, xa, xb, I0, J0, c, c == c0, c == c1);
    st = st == S - 1 ? 0 : st + 1;
  }
  // No LDS DMA may still be writing when the stages are reused or freed.
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");

  mfma_epilogue<Sh, FULL>(acc, bits, N, W, BI, BJ, I0, J0, kmax, rb_stats, lds_hist);
}

// Tile order: XCD-grouped super-tiles (grouped != 0) where the matrix is
// large enough that the L2 sharing pays, plain longest-first otherwise: with
// few 8x8 super-tiles per XCD their uneven sizes leave XCDs idle (2D
// N = 8192: 0.117 ms grouped, 0.071 ms longest-first; N = 65536: 15.2 ms
// grouped, 15.9 ms longest-first).
constexpr int64_t kGroupedMinBlocks = 129;

template <bool FULL, bool FP4>
__global__ __launch_bounds__(Big::Threads, 1) void k_count_mfma_lds(
    const uint64_t* __restrict__ bits, int64_t N, int64_t W, int64_t nb,
    int kmax, uint64_t* __restrict__ rb_stats, int grouped) {
  extern __shared__ __align__(16) char smem[];  // kStages stages, then (FULL) the bins
  uint32_t* lds_hist = (uint32_t*)(smem + kStages * Big::StageBytes);
  int64_t BI, BJ;
  if (grouped) {
    if (!tile_xcd_grouped((int64_t)blockIdx.x, nb, &BI, &BJ)) return;  // whole workgroup
  } else {
    tri_tile_longest_first((int64_t)blockIdx.x, nb, &BI, &BJ);
  }
  if constexpr (FULL) {
    const int lb = kmax + 1 < kLdsBins ? kmax + 1 : kLdsBins;
    for (int b = threadIdx.x; b < lb; b += Big::Threads) lds_hist[b] = 0;
    __syncthreads();
  }
  mfma_tile_lds<Big, FULL, FP4>(bits, N, W, BI, BJ, kmax, rb_stats, lds_hist, smem);
}

// Batched, persistent: each workgroup takes (set, BI, BJ) items of its tile
// shape, sorted longest first, in snake order until none is left.  fp4 is
// exact for the batch's N <= CS_BATCH_NMAX < 2^24.
//
// The chunks of all the workgroup's items form one stream: the LDS-DMA loads
// run kStages-1 chunks ahead of the contraction across item boundaries, so
// an item's first chunks are already in LDS when the previous item's
// epilogue runs, and the epilogue reads no memory (its relation words come
// from the item's first chunk in LDS).  The wait before chunk p is the same as in
// a single tile: at most L*(kStages-2) of the wave's vector-memory operations
// outstanding; the epilogue's loads and atomics are vector-memory
// operations too, issued after the loads they follow, and operations
// complete in issue order, so they can only make a wait longer.  At the end
// of the stream the last chunk is loaded again into a stage nobody reads
// (as the single-tile prologue does), so the count of loads in flight stays
// the same.
template <class Sh, int S>
__device__ __forceinline__ void batch_count_mfma(const BatchDev& b, const uint64_t* items, int64_t n,
                                                 char* smem) {
  constexpr int BT = Sh::BT, TM = Sh::TM, TN = Sh::TN, WN = Sh::WN, L = Sh::L;
  static_assert(L * Sh::Threads == 4 * BT && S >= 2 && L * (S - 2) <= 63, "bad stage shape");
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int r32 = lane & 31, g = lane >> 5;

  uint32_t aoff[TM], boff[TN];
#pragma unroll
  for (int t = 0; t < TM; ++t) aoff[t] = 16u * stage_slot((wave / WN) * (32 * TM) + 32 * t + r32, g);
#pragma unroll
  for (int t = 0; t < TN; ++t) boff[t] = 16u * stage_slot(BT + (wave % WN) * (32 * TN) + 32 * t + r32, g);

  typedef __attribute__((address_space(3))) void* lds_ptr;
  typedef __attribute__((address_space(1))) const void* global_ptr;

  // issue cursor: item round ki, next chunk ci of that item (last chunk ci1)
  int64_t ki = 0, ci = 0, ci1 = 0;
  bool iend = false;
  const char* gbase[L];
  uint32_t goff[L];
  auto issue_item = [&]() -> bool {
    const int64_t it = snake_item(ki);
    if (it >= n) return false;
    int64_t set, BI, BJ;
    unpack_item(items[it], &set, &BI, &BJ);
    const BatchSet bs = b.sets[set];
    const uint64_t* bits = b.bits + bs.bits_off;
    // DMA slot geometry as in mfma_tile_lds
#pragma unroll
    for (int p = 0; p < L; ++p) {
      const int slot0 = (wave * L + p) * 64;  // uniform
      const int slot = slot0 + lane;
      const int r = (slot >> 1) & (BT - 1);
      const int half = (slot & 1) ^ stage_swz(r);
      const int64_t blk = slot0 >= 2 * BT ? BJ : BI;
      gbase[p] = (const char*)(bits + blk * BT * bs.W);
      const bool valid = blk * BT + r < bs.N;
      goff[p] = (uint32_t)((valid ? (int64_t)r * bs.W * 8 : 0) + 16 * half);
    }
    ci = BI * BT / 256;
    ci1 = (BJ * BT + BT - 1) / 256;
    return true;
  };
  auto issue_next = [&](int st) {
#pragma unroll
    for (int p = 0; p < L; ++p)
      __builtin_amdgcn_global_load_lds((global_ptr)(gbase[p] + ci * 32 + goff[p]),
                                       (lds_ptr)(smem + st * Sh::StageBytes + (wave * L + p) * 1024),
                                       16, 0, 0);
    if (ci < ci1) {
      ++ci;
    } else if (!iend) {
      ++ki;
      if (!issue_item()) iend = true;  // the stream's last chunk is issued again from now on
    }
  };

  if (!issue_item()) return;  // no item for this workgroup (uniform)
#pragma unroll
  for (int k = 0; k < S - 1; ++k) issue_next(k);

  using Acc = v16f;
  int st = 0;
  for (int64_t kc = 0;; ++kc) {
    const int64_t it = snake_item(kc);
    if (it >= n) break;
    int64_t set, BI, BJ;
    unpack_item(items[it], &set, &BI, &BJ);
    const BatchSet bs = b.sets[set];
    const uint64_t* bits = b.bits + bs.bits_off;
    const int64_t I0 = BI * BT + (wave / WN) * (32 * TM);
    const int64_t J0 = BJ * BT + (wave % WN) * (32 * TN);
    Acc acc[TM][TN];
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
      for (int bb = 0; bb < TN; ++bb)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[a][bb][v] = 0;
    const int64_t c0 = BI * BT / 256, c1 = (BJ * BT + BT - 1) / 256;
    // The epilogue's relation words (bit i of row j) lie in the item's first
    // chunk of the B rows: taken from LDS there instead of from memory, whose
    // loads would wait behind the next item's chunks in flight.
    // Kept in this wave's slice of LDS past the stages until the epilogue.
    char* rel = smem + S * Sh::StageBytes + wave * (64 * TN * 16);
    // one chunk; the item's first also keeps the relation words in LDS
    auto step = [&](int64_t c, auto first) {
      asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)\n\ts_barrier" ::"n"(L * (S - 2)) : "memory");
      issue_next(st == 0 ? S - 1 : st - 1);
      const char* sb = smem + st * Sh::StageBytes;
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
      if constexpr (decltype(first)::value) {
        // keep this lane's 16 bytes of each B row (words 4c0 + 2g and
        // 4c0 + 2g + 1) for the epilogue
#pragma unroll
        for (int t = 0; t < TN; ++t)
          *(uint4*)(rel + (t * 64 + lane) * 16) = make_uint4(xb[t][0], xb[t][1], xb[t][2], xb[t][3]);
      }
      mfma_chunk<Sh, true>(acc, xa, xb, I0, J0, c, c == c0, c == c1);
      st = st == S - 1 ? 0 : st + 1;
    };
    step(c0, std::true_type{});
    for (int64_t c = c0 + 1; c <= c1; ++c) step(c, std::false_type{});
    mfma_epilogue<Sh, false>(acc, bits, bs.N, bs.W, BI, BJ, I0, J0, 3, b.stats + bs.stats_off, nullptr, rel,
                             (int)((I0 >> 6) - 4 * c0));
  }
  // No LDS DMA may still be writing when the workgroup ends.
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

// LDS of a batched count workgroup: S stages, then each wave's relation words.
// Stages of the batched kernels (4/4, 4/5, 5/6 and 6/8 for the 256- and
// 128-row tiles gave the same 512-set ensemble time within 5%).
constexpr int kBatchStagesBig = 4;
constexpr int kBatchStagesSmall = 4;
template <class Sh, int S>
constexpr int batch_lds_bytes() {
  return S * Sh::StageBytes + (Sh::Threads / 64) * 64 * Sh::TN * 16;
}
constexpr int kBatchLdsBig = batch_lds_bytes<Big, kBatchStagesBig>();
constexpr int kBatchLdsSmall = batch_lds_bytes<Small, kBatchStagesSmall>();

__global__ __launch_bounds__(Big::Threads, 1) void k_batch_count_mfma(BatchDev b) {
  extern __shared__ __align__(16) char smem[];  // kBatchLdsBig bytes
  batch_count_mfma<Big, kBatchStagesBig>(b, b.mfma_items, b.n_mfma, smem);
}

// 128-row tiles: at least 3 waves per SIMD (three workgroups per CU), so one
// workgroup's prologue and epilogue overlap the others' matrix-core work.
__global__ __launch_bounds__(Small::Threads) __attribute__((amdgpu_waves_per_eu(3, 8))) void
k_batch_count_mfma128(BatchDev b) {
  extern __shared__ __align__(16) char smem[];  // kBatchLdsSmall bytes
  batch_count_mfma<Small, kBatchStagesSmall>(b, b.mfma128_items, b.n_mfma128, smem);
}

// 128-row tiles for one set (N_0..N_3): a workgroup of 4 waves, three per CU.
constexpr int64_t kSmallTileMaxN = 4096;
template <bool FP4>
__global__ __launch_bounds__(Small::Threads) __attribute__((amdgpu_waves_per_eu(3, 8))) void
k_count_mfma_lds128(const uint64_t* __restrict__ bits, int64_t N, int64_t W, int64_t nb, int kmax,
                    uint64_t* __restrict__ rb_stats) {
  __shared__ __align__(16) char smem[kStages * Small::StageBytes];
  int64_t BI, BJ;
  tri_tile_longest_first((int64_t)blockIdx.x, nb, &BI, &BJ);
  mfma_tile_lds<Small, false, FP4>(bits, N, W, BI, BJ, kmax, rb_stats, nullptr, smem);
}

template <bool FP4>
hipError_t launch_count(const uint64_t* bits, int64_t N, int64_t W, int kmax,
                        uint64_t* rb_stats, hipStream_t st) {
  static_assert(Big::BT == kRowBlock, "block tile must equal the stats row block");
  if (N <= 1) return hipSuccess;
  // Small sets: 128-row tiles, three workgroups per CU (2D N = 1024: 0.052 ms
  // against 0.059 ms with 256-row tiles; no gain by N = 8192, a loss at 32768)
  if constexpr (FP4) {
    if (kmax <= 3 && N <= kSmallTileMaxN) {
      const int64_t nb128 = (N + Small::BT - 1) / Small::BT;
      hipLaunchKernelGGL((k_count_mfma_lds128<FP4>), dim3((unsigned)(nb128 * (nb128 + 1) / 2)),
                         dim3(Small::Threads), 0, st, bits, N, W, nb128, kmax, rb_stats);
      return hipGetLastError();
    }
  }
  const int64_t nb = (N + Big::BT - 1) / Big::BT;
  const int grouped = nb >= kGroupedMinBlocks ? 1 : 0;
  const int64_t ntiles = grouped ? xcd_grouped_ids(nb) : nb * (nb + 1) / 2;
  if (ntiles > 0x7fffffffLL) return hipErrorInvalidValue;
  const size_t stage_bytes = (size_t)kStages * Big::StageBytes;
  if (kmax <= 3) {
    hipLaunchKernelGGL((k_count_mfma_lds<false, FP4>), dim3((unsigned)ntiles), dim3(Big::Threads),
                       stage_bytes, st, bits, N, W, nb, kmax, rb_stats, grouped);
  } else {
    const size_t lds = stage_bytes + (size_t)(kmax + 1 < kLdsBins ? kmax + 1 : kLdsBins) * sizeof(uint32_t);
    hipLaunchKernelGGL((k_count_mfma_lds<true, FP4>), dim3((unsigned)ntiles), dim3(Big::Threads), lds,
                       st, bits, N, W, nb, kmax, rb_stats, grouped);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_count_mfma(const uint64_t* bits, int64_t N, int64_t W, int kmax,
                             uint64_t* rb_stats, hipStream_t st) {
  return launch_count<false>(bits, N, W, kmax, rb_stats, st);
}

hipError_t launch_count_mfma_fp4(const uint64_t* bits, int64_t N, int64_t W, int kmax,
                                 uint64_t* rb_stats, hipStream_t st) {
  return launch_count<true>(bits, N, W, kmax, rb_stats, st);
}

// Dynamic LDS limits of the staged kernels (above the 64 KiB default).
hipError_t init_count_mfma() {
  const int stages = kStages * Big::StageBytes;
  const int full = stages + kLdsBins * (int)sizeof(uint32_t);
  hipError_t e = hipFuncSetAttribute((const void*)k_batch_count_mfma,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, kBatchLdsBig);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_batch_count_mfma128, hipFuncAttributeMaxDynamicSharedMemorySize,
                            kBatchLdsSmall);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_count_mfma_lds<false, false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, stages);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_count_mfma_lds<false, true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, stages);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_count_mfma_lds<true, false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, full);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_count_mfma_lds<true, true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, full);
  return e;
}

hipError_t launch_batch_count_mfma(const BatchDev& b, int grid, hipStream_t st) {
  if (b.n_mfma <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_count_mfma, dim3((unsigned)grid), dim3(Big::Threads),
                     (size_t)kBatchLdsBig, st, b);
  return hipGetLastError();
}

hipError_t launch_batch_count_mfma128(const BatchDev& b, int grid, hipStream_t st) {
  if (b.n_mfma128 <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_count_mfma128, dim3((unsigned)grid), dim3(Small::Threads),
                     (size_t)kBatchLdsSmall, st, b);
  return hipGetLastError();
}

int batch_count_max_blocks(int kind) {
  // resident workgroups per CU of the batched count kernels
  if (kind == 1) return batch_count_pop_max_blocks();
  int n = 0;
  hipError_t e = hipSuccess;
  if (kind == 2)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (const void*)k_batch_count_mfma,
                                                     Big::Threads, (size_t)kBatchLdsBig);
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (const void*)k_batch_count_mfma128,
                                                     Small::Threads, (size_t)kBatchLdsSmall);
  return e == hipSuccess && n > 0 ? n : 1;
}

}  // namespace cs
