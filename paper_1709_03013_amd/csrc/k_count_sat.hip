// k_count_sat.hip -- local abundances N_0..N_3 and R by a saturating count.
//
// Eq. 4 (and its 4D counterpart) needs only the related pairs whose interval
// holds at most three elements (Sec. 1.2).  A pair's count can therefore stop
// as soon as it reaches 4: the exact m is still found for every pair with
// m <= 3, and every other pair is only known to have m >= 4.  The result,
// N_0..N_3 and R, is identical to the full count's (Sec. 4.1 definition).
//
// gfx950 design: one 256-thread workgroup per 64x64 tile of pairs (rows of
// block bi against rows of block bj >= bi; word bi of a row holds the columns
// of block bi), so the interval of every pair of the tile lies in words
// bi..bj.
//  1. A window of at most kSatWin words of the 128 rows is staged in LDS
//     (all loads issued before the first wait), with the interval masks
//     applied while staging: word bi of row i keeps columns above i, word bj
//     of row j columns below j.
//  2. Dense step: all 4096 pairs count the C words in the middle of the gap
//     between the blocks (register-blocked AND + popcount, 4x4 pairs per
//     thread).  A pair's interior elements are spread over its whole label
//     range, and its middle is where most of them lie.  Tiles whose words
//     bi..bj fit in C+2 words count all of them here and are done.
//  3. Related pairs still below 4 stay pending in their thread's registers
//     and are taken, one at a time, by the thread's 16-lane group: one step
//     over the rest of the staged window (one word per lane, outward from
//     the chunk), then, for the few still below 4, steps of 16 words
//     upward and 16 downward read from HBM (128-byte row segments, two words
//     per lane) until the count reaches 4 or the pair's words are exhausted.
// There is no global queue or counter: a tile finishes its own pairs, and
// its counts go to its row block's slot with one atomic add per counter.
#include "cs_device.h"
#include "cs_internal.h"

namespace cs {

namespace {

constexpr int kStride = kSatWin + 1;  // odd row stride: conflict-free 64-bit LDS reads

__device__ __forceinline__ uint32_t popc64(uint64_t x) {
  return bcnt_acc((uint32_t)(x >> 32), bcnt_acc((uint32_t)x, 0u));
}

__device__ __forceinline__ uint64_t above(int r) { return ~((2ull << r) - 1); }  // columns > r
__device__ __forceinline__ uint64_t below(int r) { return (1ull << r) - 1; }     // columns < r

// Sum over the 16 lanes of a group (lanes 16g..16g+15 of the wave).
__device__ __forceinline__ uint32_t group_sum16(uint32_t p) {
  p += __shfl_xor(p, 1, 16);
  p += __shfl_xor(p, 2, 16);
  p += __shfl_xor(p, 4, 16);
  p += __shfl_xor(p, 8, 16);
  return p;
}

// Continue one pair from HBM with its 16-lane group: words of [bi, bj]
// outside the staged window [w0, w1), lanes 0-7 upward from w1 and lanes
// 8-15 downward from w0, kFinishWords consecutive words per lane per step
// (independent loads, one memory latency per step), until the count reaches
// 4.  c is uniform across the group, so every lane leaves the loop in the
// same iteration.
constexpr int kFinishWords = 2;

__device__ __forceinline__ uint32_t finish_group(const uint64_t* __restrict__ bits, int64_t W,
                                                 int64_t i, int64_t j, int64_t bi, int64_t bj,
                                                 int64_t w0, int64_t w1, uint32_t c, int l) {
  const uint64_t* ri = bits + i * W;
  const uint64_t* rj = bits + j * W;
  const uint64_t mi = above((int)(i & 63)), mj = below((int)(j & 63));
  const bool upward = l < 8;
  const int64_t lo = (int64_t)(upward ? l : l - 8) * kFinishWords;
  int64_t up = w1, dn = w0;
  while (c < 4 && (up <= bj || dn > bi)) {
    uint32_t p = 0;
#pragma unroll
    for (int u = 0; u < kFinishWords; ++u) {
      const int64_t w = upward ? up + lo + u : dn - 1 - lo - u;
      if (upward ? w <= bj : w >= bi) {
        uint64_t a = ri[w], b = rj[w];
        if (w == bi) a &= mi;
        if (w == bj) b &= mj;
        p += popc64(a & b);
      }
    }
    c += group_sum16(p);
    up += 8 * kFinishWords;
    dn -= 8 * kFinishWords;
  }
  return c;
}

__device__ __forceinline__ void add_block(uint64_t* __restrict__ blk, int64_t b, const uint32_t* v,
                                          int n) {
  for (int k = 0; k < n; ++k)
    if (v[k]) atomicAdd((unsigned long long*)&blk[b * kSatBlkWords + k], (unsigned long long)v[k]);
}

__global__ __launch_bounds__(256) void k_sat_tile(const uint64_t* __restrict__ bits, int64_t N,
                                                  int64_t W, int64_t nb, int C, int E,
                                                  uint64_t* __restrict__ blk) {
  __shared__ uint64_t sI[64 * kStride];
  __shared__ uint64_t sJ[64 * kStride];
  __shared__ uint64_t srel[64];
  __shared__ uint32_t red[4][6];

  int64_t bi, bj;
  if (!tile_xcd_grouped((int64_t)blockIdx.x, nb, &bi, &bj)) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const SatWin win = sat_window(bi, bj, C, E);
  const int nw = (int)(win.w1 - win.w0);

  // issue every global load of the tile before the first wait: the relation
  // word of each I row (bit jl of srel[il]: 64bi+il related to 64bj+jl) and
  // the window, thread (r, q) taking words q, q+4, ... of I row r and J row r
  const int r = tid >> 2, q = tid & 3;
  const int64_t ri = bi * 64 + r, rj = bj * 64 + r;
  uint64_t relv = 0, va[kSatWin / 4], vb[kSatWin / 4];
  if (tid < 64 && bi * 64 + tid < N) relv = bits[(bi * 64 + tid) * W + bj];
  {
    const uint64_t* pi = bits + (ri < N ? ri : 0) * W + win.w0;
    const uint64_t* pj = bits + (rj < N ? rj : 0) * W + win.w0;
#pragma unroll
    for (int t = 0; t < kSatWin / 4; ++t) {
      const int k = q + 4 * t;
      va[t] = (k < nw && ri < N) ? pi[k] : 0ull;
      vb[t] = (k < nw && rj < N) ? pj[k] : 0ull;
    }
  }
  if (tid < 64) srel[tid] = relv;
#pragma unroll
  for (int t = 0; t < kSatWin / 4; ++t) {
    const int k = q + 4 * t;
    if (k < nw) {
      const int64_t w = win.w0 + k;
      sI[r * kStride + k] = w == bi ? (va[t] & above(r)) : va[t];
      sJ[r * kStride + k] = w == bj ? (vb[t] & below(r)) : vb[t];
    }
  }
  __syncthreads();
  if (!__syncthreads_or(srel[tid & 63] != 0ull)) return;  // no related pair in the tile

  // dense chunk: thread (ti, tj) owns rows ti+16a and columns tj+16b
  const int ti = tid >> 4, tj = tid & 15;
  const int k0 = (int)(win.c0 - win.w0), k1 = (int)(win.c1 - win.w0);
  uint32_t acc[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) acc[t] = 0;
  for (int k = k0; k < k1; ++k) {
    uint64_t x[4], y[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) x[a] = sI[(ti + 16 * a) * kStride + k];
#pragma unroll
    for (int b = 0; b < 4; ++b) y[b] = sJ[(tj + 16 * b) * kStride + k];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const uint64_t v = x[a] & y[b];
        acc[4 * a + b] = bcnt_acc((uint32_t)(v >> 32), bcnt_acc((uint32_t)v, acc[4 * a + b]));
      }
  }

  // classify: related pairs below 4 are final if the chunk covered their
  // whole interval; otherwise this thread marks them pending (bit 4a+b of
  // pend) with their count so far (bits 2(4a+b) of pc)
  const bool chunk_all = win.c0 == bi && win.c1 == bj + 1;
  const bool window_all = win.w0 == bi && win.w1 == bj + 1;
  uint32_t cnt[6] = {0, 0, 0, 0, 0, 0};  // N_0..N_3, R, pairs continued from HBM
  uint32_t pend = 0, pc = 0;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int il = ti + 16 * a;
    const uint64_t rw = srel[il];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int jl = tj + 16 * b;
      const bool rel = ((rw >> jl) & 1ull) && (bi < bj || il < jl);
      const uint32_t m = acc[4 * a + b];
      cnt[4] += rel ? 1u : 0u;
      if (rel && m < 4) {
        if (chunk_all) {
          cnt[0] += m == 0; cnt[1] += m == 1; cnt[2] += m == 2; cnt[3] += m == 3;
        } else {
          pend |= 1u << (4 * a + b);
          pc |= m << (2 * (4 * a + b));
        }
      }
    }
  }

  if (!chunk_all) {
    // The 16 threads tid = 16ti + tj (tj = 0..15) form a group; it takes
    // its threads' pending pairs one at a time (lowest lane first); lane l
    // adds the staged words l, l+16, ... of those outside the chunk.  Every
    // pass clears one pending bit, so the loop ends after at most 256
    // passes; its exit is uniform in the group.
    const int l = tj, gbase = lane & 48;
    const int nup = nw - k1, nout = k0 + nup;  // staged words outside the chunk
    for (;;) {
      const uint32_t gm = (uint32_t)(__ballot(pend != 0) >> gbase) & 0xffffu;
      if (!gm) break;
      const int src = __builtin_ctz(gm);
      const uint32_t sp = __shfl(pend, gbase + src, 64);
      const uint32_t spc = __shfl(pc, gbase + src, 64);
      const int qb = __builtin_ctz(sp);
      if (l == src) pend &= pend - 1;
      const int il = ti + 16 * (qb >> 2), jl = src + 16 * (qb & 3);
      uint32_t c = (spc >> (2 * qb)) & 3u;
      uint32_t p = 0;
      for (int o = l; o < nout; o += 16) {
        const int k = o < nup ? k1 + o : k0 - 1 - (o - nup);
        p += popc64(sI[il * kStride + k] & sJ[jl * kStride + k]);
      }
      c += group_sum16(p);
      if (c < 4 && !window_all) {
        cnt[5] += l == 0;
        c = finish_group(bits, W, bi * 64 + il, bj * 64 + jl, bi, bj, win.w0, win.w1, c, l);
      }
      if (c < 4 && l == 0) {
        cnt[0] += c == 0; cnt[1] += c == 1; cnt[2] += c == 2; cnt[3] += c == 3;
      }
    }
  }

  // tile totals -> the row block's counters (each at most the tile's 4096
  // pairs, so two share a 32-bit word through the wave sum)
#pragma unroll
  for (int k = 0; k < 6; k += 2) {
    const uint32_t t = wave_total_u32(cnt[k] | (cnt[k + 1] << 16));
    cnt[k] = t & 0xFFFFu;
    cnt[k + 1] = t >> 16;
  }
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < 6; ++k) red[wave][k] = cnt[k];
  __syncthreads();
  if (tid == 0) {
    uint32_t t[6];
    for (int k = 0; k < 6; ++k) t[k] = red[0][k] + red[1][k] + red[2][k] + red[3][k];
    add_block(blk, bi, t, 6);
  }
}

// Sum the per-block counters: out[k] = sum over blocks of blk[b][k], k < 6.
__global__ __launch_bounds__(256) void k_sat_reduce(const uint64_t* __restrict__ blk, int64_t nb,
                                                    uint64_t* __restrict__ out) {
  __shared__ uint64_t part[256];
  const int col = blockIdx.x;
  uint64_t s = 0;
  for (int64_t b = threadIdx.x; b < nb; b += 256) s += blk[b * kSatBlkWords + col];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[col] = part[0];
}

}  // namespace

uint64_t sat_workspace_bytes(int64_t N) {
  const int64_t nb = (N + 63) / 64;
  return (uint64_t)(nb > 0 ? nb : 1) * kSatBlkWords * 8;
}

hipError_t launch_count_sat(const uint64_t* bits, int64_t N, int64_t W, int C, int E,
                            uint64_t* blk, uint64_t* out, hipStream_t st) {
  const int64_t nb = (N + 63) / 64;
  hipError_t e = launch_fill_u64(blk, 0, (size_t)(nb > 0 ? nb : 1) * kSatBlkWords, st);
  if (e != hipSuccess) return e;
  if (N >= 2) {
    const int64_t ids = xcd_grouped_ids(nb);
    if (ids > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sat_tile, dim3((unsigned)ids), dim3(256), 0, st, bits, N, W, nb, C, E,
                       blk);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_sat_reduce, dim3(6), dim3(256), 0, st, blk, nb > 0 ? nb : 1, out);
  return hipGetLastError();
}

}  // namespace cs
