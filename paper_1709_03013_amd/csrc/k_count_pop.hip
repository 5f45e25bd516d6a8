// k_count_pop.hip -- interval counting on the vector ALU (Sec. 4.3, Alg. 5,
// Fig. 2): for every related pair i<j, m = popcount(row_i AND row_j) over
// columns i+1..j-1, then the histogram of m.
//
// gfx950 design: the paper's partial vector product, register-blocked the
// way a VALU GEMM is.  One wave (one workgroup) owns a 64x64 tile of pairs:
// rows i in block bi, rows j in block bj >= bi (64 labels per block).  Its
// 64 lanes form an 8x8 grid; lane (li, lj) accumulates the 8x8 pairs
// i = 64bi + 8li + a, j = 64bj + 8lj + b in 64 registers.  The words bi..bj
// of the 64+64 rows stream through LDS in chunks of four (word-major, so a
// lane's 8 rows of one word are one 64-byte read, broadcast to the 8 lanes
// that share them); each pair then costs 2x v_and_b32 + 2x v_bcnt_u32_b32
// per 64-bit word, all operands in VGPRs.  The interval mask is applied once,
// while staging: word bi of row i keeps only columns above i, word bj of row
// j only columns below j; words outside [bi, bj] are zero.
// Unrelated pairs and pairs with i >= j are computed too and dropped at the
// end by the relation bit (bit j of row i, word bj).  Histogram counters,
// R and the sum of m are reduced across the wave with shuffles and added to
// the tile's row-block stats with one atomic each.
//
// Tiles run longest-first (decreasing bj - bi) to shorten the tail.
#include "cs_device.h"
#include "cs_internal.h"

namespace cs {
namespace {

constexpr int kChunk = 4;  // words per staging step (rows are 4-word aligned)

// One 64x64 tile of pairs (rows of block bi against rows of block bj >= bi)
// by one 64-lane workgroup.  sI, sJ: word-major staging, sI[k][r] = word
// (w+k) of row 64bi+r.  lds_hist (FULL only) holds min(kmax+1, kLdsBins)
// zeroed bins; larger sizes go straight to the row-block stats.
template <bool FULL>
__device__ __forceinline__ void pop_tile(const uint64_t* __restrict__ bits, int64_t N,
                                         int64_t W, int64_t bi, int64_t bj, int kmax,
                                         uint64_t* __restrict__ rb_stats,
                                         uint32_t* lds_hist, uint64_t (*sI)[64],
                                         uint64_t (*sJ)[64]) {
  const int lane = threadIdx.x;
  const int li = lane >> 3, lj = lane & 7;

  // Staging rows of this lane: I row 64bi+lane and J row 64bj+lane.
  const int64_t ri = bi * 64 + lane, rj = bj * 64 + lane;
  const bool ri_ok = ri < N, rj_ok = rj < N;
  const uint64_t* pi = bits + (ri_ok ? ri : 0) * W;
  const uint64_t* pj = bits + (rj_ok ? rj : 0) * W;
  const uint64_t mask_above = ~((2ull << lane) - 1);  // columns > ri
  const uint64_t mask_below = (1ull << lane) - 1;     // columns < rj

  uint32_t acc[64];
#pragma unroll
  for (int q = 0; q < 64; ++q) acc[q] = 0;

  const int64_t w_first = bi & ~(int64_t)(kChunk - 1);
  uint64_t xi[kChunk], xj[kChunk];
#pragma unroll
  for (int k = 0; k < kChunk; ++k) {
    xi[k] = pi[w_first + k];
    xj[k] = pj[w_first + k];
  }
  for (int64_t w = w_first; w <= bj; w += kChunk) {
    __syncthreads();  // previous chunk fully consumed
#pragma unroll
    for (int k = 0; k < kChunk; ++k) {
      const int64_t wk = w + k;
      uint64_t a = (ri_ok && wk >= bi && wk <= bj) ? xi[k] : 0ull;
      a = (wk == bi) ? (a & mask_above) : a;
      uint64_t b = rj_ok ? xj[k] : 0ull;
      b = (wk == bj) ? (b & mask_below) : b;
      sI[k][lane] = a;
      sJ[k][lane] = b;
    }
    __syncthreads();
    // prefetch the next chunk while this one is counted
    if (w + kChunk <= bj) {
#pragma unroll
      for (int k = 0; k < kChunk; ++k) {
        xi[k] = pi[w + kChunk + k];
        xj[k] = pj[w + kChunk + k];
      }
    }
#pragma unroll
    for (int k = 0; k < kChunk; ++k) {
      uint64_t iw[8], jw[8];
#pragma unroll
      for (int a = 0; a < 8; ++a) iw[a] = sI[k][8 * li + a];
#pragma unroll
      for (int b = 0; b < 8; ++b) jw[b] = sJ[k][8 * lj + b];
#pragma unroll
      for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int b = 0; b < 8; ++b) {
          const uint64_t x = iw[a] & jw[b];
          uint32_t c = acc[8 * a + b];
          c = bcnt_acc((uint32_t)x, c);
          c = bcnt_acc((uint32_t)(x >> 32), c);
          acc[8 * a + b] = c;
        }
    }
  }

  // Epilogue: relation bits of this lane's 8 rows against its 8 columns.
  uint32_t cnt[4] = {0, 0, 0, 0};
  uint32_t nrel = 0;
  uint64_t summ = 0;
  uint64_t* st = rb_stats + ((bi * 64) / kRowBlock) * (int64_t)(kmax + 3);
  const uint32_t lb = (uint32_t)(kmax + 1 < kLdsBins ? kmax + 1 : kLdsBins);
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const int64_t i = bi * 64 + 8 * li + a;
    const uint64_t relw = i < N ? bits[i * W + bj] : 0ull;
    const uint32_t rbyte = (uint32_t)(relw >> (8 * lj)) & 0xffu;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool valid = ((rbyte >> b) & 1u) && (bi < bj || 8 * li + a < 8 * lj + b);
      const uint32_t m = acc[8 * a + b];
      nrel += valid ? 1u : 0u;
      summ += valid ? m : 0u;
      if constexpr (FULL) {
        if (valid && m <= (uint32_t)kmax) {
          if (m < lb) atomicAdd(&lds_hist[m], 1u);
          else atomicAdd((unsigned long long*)&st[m], 1ull);
        }
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) cnt[k] += (valid && m == (uint32_t)k) ? 1u : 0u;
      }
    }
  }
  nrel = wave_sum_u32(nrel);
  summ = wave_sum_u64(summ);
  if constexpr (!FULL) {
#pragma unroll
    for (int k = 0; k < 4; ++k) cnt[k] = wave_sum_u32(cnt[k]);
    if (lane < 4) {
      const uint32_t v = lane == 0 ? cnt[0] : lane == 1 ? cnt[1] : lane == 2 ? cnt[2] : cnt[3];
      if (v) atomicAdd((unsigned long long*)&st[lane], (unsigned long long)v);
    }
  } else {
    __syncthreads();
    for (int b = lane; b < (int)lb; b += 64) {
      const uint32_t v = lds_hist[b];
      if (v) atomicAdd((unsigned long long*)&st[b], (unsigned long long)v);
    }
  }
  if (lane == 0) {
    if (nrel) atomicAdd((unsigned long long*)&st[kmax + 1], (unsigned long long)nrel);
    if (summ) atomicAdd((unsigned long long*)&st[kmax + 2], (unsigned long long)summ);
  }
}

// One tile per workgroup.  N_0..N_3: at least 3 waves per SIMD (the
// accumulators and operands fit in 168 registers); the full histogram's
// epilogue needs more registers and runs at 2.
template <bool FULL>
__device__ __forceinline__ void count_pop_tile(const uint64_t* __restrict__ bits, int64_t N,
                                               int64_t W, int64_t nb, int kmax,
                                               uint64_t* __restrict__ rb_stats) {
  __shared__ uint64_t sI[kChunk][64];
  __shared__ uint64_t sJ[kChunk][64];
  extern __shared__ uint32_t lds_hist[];  // FULL only: min(kmax+1, kLdsBins) bins
  int64_t bi, bj;
  tri_tile_longest_first((int64_t)blockIdx.x, nb, &bi, &bj);
  if constexpr (FULL) {
    const int lb = kmax + 1 < kLdsBins ? kmax + 1 : kLdsBins;
    for (int b = threadIdx.x; b < lb; b += 64) lds_hist[b] = 0;
  }
  pop_tile<FULL>(bits, N, W, bi, bj, kmax, rb_stats, lds_hist, sI, sJ);
}

__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_count_pop(
    const uint64_t* __restrict__ bits, int64_t N, int64_t W, int64_t nb,
    int kmax, uint64_t* __restrict__ rb_stats) {
  count_pop_tile<false>(bits, N, W, nb, kmax, rb_stats);
}

__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 8))) void k_count_pop_full(
    const uint64_t* __restrict__ bits, int64_t N, int64_t W, int64_t nb,
    int kmax, uint64_t* __restrict__ rb_stats) {
  count_pop_tile<true>(bits, N, W, nb, kmax, rb_stats);
}

// Batched, persistent: each 64-lane workgroup takes (set, bi, bj) items,
// sorted longest first, in snake order until none is left.  The item loop
// and the set table need registers beyond the single-tile kernel's 168.
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 8))) void k_batch_count_pop(
    BatchDev b) {
  __shared__ uint64_t sI[kChunk][64];
  __shared__ uint64_t sJ[kChunk][64];
  for (int64_t k = 0;; ++k) {
    const int64_t it = snake_item(k);
    if (it >= b.n_pop) break;
    int64_t set, bi, bj;
    unpack_item(b.pop_items[it], &set, &bi, &bj);
    const BatchSet bs = b.sets[set];
    pop_tile<false>(b.bits + bs.bits_off, bs.N, bs.W, bi, bj, 3, b.stats + bs.stats_off,
                    nullptr, sI, sJ);
  }
}

// Batched epilogue: one workgroup per set sums its row-block stats and
// evaluates the BD action (same integer bracket and single rounding as the
// single-set path).
__global__ __launch_bounds__(256) void k_batch_finish(BatchDev b) {
  __shared__ uint64_t part[6][256];
  const int s = blockIdx.x;
  const BatchSet bs = b.sets[s];
  const int64_t nrb = (bs.N + kRowBlock - 1) / kRowBlock;
  uint64_t acc[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t r = threadIdx.x; r < nrb; r += 256)
    for (int c = 0; c < 6; ++c) acc[c] += b.stats[bs.stats_off + r * 6 + c];
  for (int c = 0; c < 6; ++c) part[c][threadIdx.x] = acc[c];
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o)
      for (int c = 0; c < 6; ++c) part[c][threadIdx.x] += part[c][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    cs_result r;
    for (int c = 0; c < 4; ++c) r.n[c] = part[c][0];
    r.R = part[4][0];
    r.summ = part[5][0];
    const int64_t N = bs.N;
    if (bs.d == 2) {
      const int64_t K = N - 2 * (int64_t)r.n[0] + 4 * (int64_t)r.n[1] - 2 * (int64_t)r.n[2];
      r.S = 2.0 * (double)K;
    } else {
      const int64_t K = N - (int64_t)r.n[0] + 9 * (int64_t)r.n[1] - 16 * (int64_t)r.n[2] +
                        8 * (int64_t)r.n[3];
      r.S = b.c4 * (double)K;
    }
    r.status = CS_OK;
    r.reserved = 0;
    b.results[s] = r;
  }
}

__global__ __launch_bounds__(256) void k_reduce_rows(
    const uint64_t* __restrict__ rb, int64_t nrb, int stride,
    uint64_t* __restrict__ tot) {
  __shared__ uint64_t part[256];
  const int col = blockIdx.x;
  uint64_t s = 0;
  for (int64_t b = threadIdx.x; b < nrb; b += 256) s += rb[b * stride + col];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) tot[col] = part[0];
}

}  // namespace

int64_t num_row_blocks(int64_t N) { return (N + kRowBlock - 1) / kRowBlock; }

hipError_t launch_count_pop(const uint64_t* bits, int64_t N, int64_t W,
                            int kmax, uint64_t* rb_stats, hipStream_t st) {
  if (N <= 1) return hipSuccess;
  const int64_t nb = (N + 63) / 64;
  const int64_t ntiles = nb * (nb + 1) / 2;
  if (ntiles > 0x7fffffffLL) return hipErrorInvalidValue;
  if (kmax <= 3) {
    hipLaunchKernelGGL(k_count_pop, dim3((unsigned)ntiles), dim3(64), 0, st,
                       bits, N, W, nb, kmax, rb_stats);
  } else {
    const size_t lds = (size_t)(kmax + 1 < kLdsBins ? kmax + 1 : kLdsBins) * sizeof(uint32_t);
    hipLaunchKernelGGL(k_count_pop_full, dim3((unsigned)ntiles), dim3(64), lds, st,
                       bits, N, W, nb, kmax, rb_stats);
  }
  return hipGetLastError();
}

hipError_t launch_batch_count_pop(const BatchDev& b, int grid, hipStream_t st) {
  if (b.n_pop <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_count_pop, dim3((unsigned)grid), dim3(64), 0, st, b);
  return hipGetLastError();
}

int batch_count_pop_max_blocks() {
  int n = 0;
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (const void*)k_batch_count_pop, 64, 0);
  return e == hipSuccess && n > 0 ? n : 1;
}

hipError_t launch_batch_finish(const BatchDev& b, hipStream_t st) {
  if (b.nsets <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_finish, dim3((unsigned)b.nsets), dim3(256), 0, st, b);
  return hipGetLastError();
}

hipError_t launch_reduce_rows(const uint64_t* rb_stats, int64_t nrb, int kmax,
                              uint64_t* tot, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_rows, dim3((unsigned)(kmax + 3)), dim3(256), 0, st,
                     rb_stats, nrb, kmax + 3, tot);
  return hipGetLastError();
}

}  // namespace cs
