// k_count_sat.hip -- local abundances N_0..N_3 and R by a saturating count.
//
// Eq. 4 (and its 4D counterpart) needs only the related pairs whose interval
// holds at most three elements (Sec. 1.2).  A pair's count can therefore stop
// as soon as it reaches 4: the exact m is still found for every pair with
// m <= 3, and every other pair is only known to have m >= 4.  The result,
// N_0..N_3 and R, is identical to the full count's (Sec. 4.1 definition).
//
// gfx950 design, two passes over the packed matrix:
//  1. k_sat_tile: one 256-thread workgroup per 64x64 tile of pairs (rows of
//     block bi against rows of block bj >= bi; word bi of a row holds the
//     columns of block bi).  The interval of every pair of the tile lies in
//     words bi..bj.  A window of at most kSatWin words of the 128 rows is
//     staged in LDS, with the interval masks applied while staging (word bi
//     of row i keeps columns above i, word bj of row j columns below j).
//     All 4096 pairs first count C words in the middle of the gap between
//     the blocks (dense, register-blocked AND + popcount, 4x4 pairs per
//     thread): a pair's interior elements are spread over its whole label
//     range, and the middle is where a pair of the tile meets most of them.
//     Related pairs still below 4 are listed in LDS and continue, one lane
//     each, over the rest of the staged window, outward from the chunk.
//     Pairs the window does not finish are appended to a queue in HBM (one
//     atomic per wave); if the queue is full the lane finishes its pair
//     itself from HBM, so the result never depends on the queue's size.
//     Tiles whose words bi..bj fit in C+2 words are counted exactly by the
//     dense step alone.
//  2. k_sat_queue: 16 lanes per queued pair, 8 words upward and 8 downward
//     per step (coalesced 64-byte row segments), until the count reaches 4
//     or the pair's words are exhausted.
// Counts go to per-row-block counters (pairs with i in block bi; one 64-byte
// slot per block) and k_sat_reduce sums them.
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

// Queue entry: i (30 bits) | count so far (2 bits) | j (32 bits).
__device__ __forceinline__ uint64_t pack_pair(int64_t i, int64_t j, uint32_t c) {
  return (uint64_t)i | ((uint64_t)c << 30) | ((uint64_t)j << 32);
}

// Finish one pair serially from HBM: words of [bi, bj] outside the staged
// window [w0, w1), upward first, stopping at 4.
__device__ uint32_t finish_pair(const uint64_t* __restrict__ bits, int64_t W, int64_t i,
                                int64_t j, int64_t bi, int64_t bj, int64_t w0, int64_t w1,
                                uint32_t c) {
  const uint64_t* ri = bits + i * W;
  const uint64_t* rj = bits + j * W;
  for (int64_t w = w1; c < 4 && w <= bj; ++w) {
    uint64_t b = rj[w];
    if (w == bj) b &= below((int)(j & 63));
    c += popc64(ri[w] & b);
  }
  for (int64_t w = w0 - 1; c < 4 && w >= bi; --w) {
    uint64_t a = ri[w];
    if (w == bi) a &= above((int)(i & 63));
    c += popc64(a & rj[w]);
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
                                                  uint64_t* __restrict__ blk,
                                                  unsigned long long* __restrict__ qcount,
                                                  uint64_t* __restrict__ queue, uint64_t qcap) {
  __shared__ uint64_t sI[64 * kStride];
  __shared__ uint64_t sJ[64 * kStride];
  __shared__ uint64_t srel[64];
  __shared__ uint16_t list[4096];
  __shared__ uint32_t nlist;
  __shared__ uint32_t red[4][5];

  int64_t bi, bj;
  if (!tile_xcd_grouped((int64_t)blockIdx.x, nb, &bi, &bj)) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const SatWin win = sat_window(bi, bj, C, E);
  const int nw = (int)(win.w1 - win.w0);

  // relation words (bit jl of srel[il]: i = 64bi+il related to j = 64bj+jl)
  if (tid < 64) {
    const int64_t i = bi * 64 + tid;
    srel[tid] = i < N ? bits[i * W + bj] : 0ull;
  }
  if (tid == 0) nlist = 0;
  __syncthreads();
  if (!__syncthreads_or(srel[tid & 63] != 0ull)) return;  // no related pair in the tile

  // stage the window of the 64 I rows and 64 J rows, masks applied
  {
    const int r = tid >> 2, q = tid & 3;
    const int64_t i = bi * 64 + r, j = bj * 64 + r;
    const uint64_t* pi = bits + (i < N ? i : 0) * W;
    const uint64_t* pj = bits + (j < N ? j : 0) * W;
    for (int k = q; k < nw; k += 4) {
      const int64_t w = win.w0 + k;
      uint64_t a = i < N ? pi[w] : 0ull;
      uint64_t b = j < N ? pj[w] : 0ull;
      if (w == bi) a &= above(r);
      if (w == bj) b &= below(r);
      sI[r * kStride + k] = a;
      sJ[r * kStride + k] = b;
    }
  }
  __syncthreads();

  // dense chunk: thread (ti, tj) owns rows ti+16a and columns tj+16b
  const int ti = tid >> 4, tj = tid & 15;
  const int k0 = (int)(win.c0 - win.w0), k1 = (int)(win.c1 - win.w0);
  uint32_t acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0;
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

  // classify: related pairs with m < 4 are final if the chunk covered their
  // whole interval, else listed for the window pass
  const bool chunk_all = win.c0 == bi && win.c1 == bj + 1;
  const bool window_all = win.w0 == bi && win.w1 == bj + 1;
  uint32_t cnt[5] = {0, 0, 0, 0, 0};  // N_0..N_3, R
  uint32_t nmine = 0;
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
          ++nmine;
        }
      }
    }
  }
  if (!chunk_all && nmine) {
    uint32_t slot = atomicAdd(&nlist, nmine);
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int il = ti + 16 * a;
      const uint64_t rw = srel[il];
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int jl = tj + 16 * b;
        const bool rel = ((rw >> jl) & 1ull) && (bi < bj || il < jl);
        const uint32_t m = acc[4 * a + b];
        if (rel && m < 4) list[slot++] = (uint16_t)((uint32_t)il | ((uint32_t)jl << 6) | (m << 12));
      }
    }
  }
  __syncthreads();

  if (!chunk_all) {
    const int n = (int)nlist;
    const int kup = nw - k1, kdn = k0;
    const int steps = kup > kdn ? kup : kdn;
    for (int e = tid; e < n; e += 256) {
      const uint32_t ent = list[e];
      const int il = ent & 63, jl = (ent >> 6) & 63;
      uint32_t c = ent >> 12;
      const uint64_t* xi = sI + il * kStride;
      const uint64_t* yj = sJ + jl * kStride;
      for (int s = 0; c < 4 && s < steps; ++s) {
        if (s < kup) c += popc64(xi[k1 + s] & yj[k1 + s]);
        if (s < kdn) c += popc64(xi[k0 - 1 - s] & yj[k0 - 1 - s]);
      }
      bool surv = false;
      if (c < 4) {
        if (window_all) {
          cnt[0] += c == 0; cnt[1] += c == 1; cnt[2] += c == 2; cnt[3] += c == 3;
        } else {
          surv = true;
        }
      }
      // survivors go to the queue, one atomic per wave
      const uint64_t sm = __ballot(surv);
      if (sm) {
        const int leader = __ffsll((unsigned long long)sm) - 1;
        unsigned long long base = 0;
        if (lane == leader) base = atomicAdd(qcount, (unsigned long long)__popcll(sm));
        base = __shfl(base, leader, 64);
        if (surv) {
          const uint64_t below_me = sm & ((1ull << lane) - 1);
          const uint64_t slot = (uint64_t)base + (uint64_t)__popcll(below_me);
          const int64_t i = bi * 64 + il, j = bj * 64 + jl;
          if (slot < qcap) {
            queue[slot] = pack_pair(i, j, c);
          } else {
            c = finish_pair(bits, W, i, j, bi, bj, win.w0, win.w1, c);
            cnt[0] += c == 0; cnt[1] += c == 1; cnt[2] += c == 2; cnt[3] += c == 3;
          }
        }
      }
    }
  }

  // tile totals -> the row block's counters
#pragma unroll
  for (int k = 0; k < 5; ++k) cnt[k] = wave_sum_u32(cnt[k]);
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < 5; ++k) red[wave][k] = cnt[k];
  __syncthreads();
  if (tid == 0) {
    uint32_t t[5];
    for (int k = 0; k < 5; ++k) t[k] = red[0][k] + red[1][k] + red[2][k] + red[3][k];
    add_block(blk, bi, t, 5);
  }
}

// Queued pairs: 16 lanes per pair; the queue is split into equal contiguous
// ranges, one per 16-lane group (a static schedule).  A group's counters are
// added to a row block's slot whenever its pairs move to another block.
__global__ __launch_bounds__(256) void k_sat_queue(const uint64_t* __restrict__ bits, int64_t W,
                                                   int C, int E, uint64_t* __restrict__ blk,
                                                   const unsigned long long* __restrict__ qcount,
                                                   const uint64_t* __restrict__ queue,
                                                   uint64_t qcap) {
  const uint64_t total = *qcount < qcap ? *qcount : qcap;
  const int l = threadIdx.x & 15;
  const uint64_t groups = (uint64_t)gridDim.x * 16;
  const uint64_t g = (uint64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
  const uint64_t per = (total + groups - 1) / groups;
  const uint64_t e0 = g * per;
  const uint64_t e1 = e0 + per < total ? e0 + per : total;
  uint32_t cnt[4] = {0, 0, 0, 0};
  int64_t cur = -1;
  for (uint64_t e = e0; e < e1; ++e) {
    const uint64_t ent = queue[e];
    const int64_t i = (int64_t)(ent & 0x3fffffffull);
    const int64_t j = (int64_t)(ent >> 32);
    uint32_t c = (uint32_t)(ent >> 30) & 3u;
    const int64_t bi = i >> 6, bj = j >> 6;
    if (bi != cur) {
      if (cur >= 0 && l == 0) add_block(blk, cur, cnt, 4);
      cnt[0] = cnt[1] = cnt[2] = cnt[3] = 0;
      cur = bi;
    }
    const SatWin win = sat_window(bi, bj, C, E);
    const uint64_t* ri = bits + i * W;
    const uint64_t* rj = bits + j * W;
    const uint64_t mi = above((int)(i & 63)), mj = below((int)(j & 63));
    int64_t up = win.w1, dn = win.w0;
    while (c < 4 && (up <= bj || dn > bi)) {
      const int64_t w = l < 8 ? up + l : dn - 1 - (l - 8);
      const bool ok = l < 8 ? w <= bj : w >= bi;
      uint32_t p = 0;
      if (ok) {
        uint64_t a = ri[w], b = rj[w];
        if (w == bi) a &= mi;
        if (w == bj) b &= mj;
        p = popc64(a & b);
      }
      p += __shfl_xor(p, 1, 16);
      p += __shfl_xor(p, 2, 16);
      p += __shfl_xor(p, 4, 16);
      p += __shfl_xor(p, 8, 16);
      c += p;
      up += 8;
      dn -= 8;
    }
    if (c < 4) ++cnt[c];
  }
  if (cur >= 0 && l == 0) add_block(blk, cur, cnt, 4);
}

// Sum the per-block counters: out[k] = sum over blocks of blk[b][k], k < 5;
// out[5] = pairs queued by the tile pass.
__global__ __launch_bounds__(256) void k_sat_reduce(const uint64_t* __restrict__ blk, int64_t nb,
                                                    const uint64_t* __restrict__ qcount,
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
  if (col == 0 && threadIdx.x == 0) out[5] = *qcount;
}

}  // namespace

uint64_t sat_workspace_bytes(int64_t N, uint64_t qcap) {
  const int64_t nb = (N + 63) / 64;
  return 256 + (uint64_t)(nb > 0 ? nb : 1) * kSatBlkWords * 8 + qcap * 8;
}

hipError_t launch_count_sat(const uint64_t* bits, int64_t N, int64_t W, int C, int E,
                            uint64_t* blk, uint64_t* qcount, uint64_t* queue, uint64_t qcap,
                            uint64_t* out, int queue_grid, hipStream_t st) {
  const int64_t nb = (N + 63) / 64;
  hipError_t e = launch_fill_u64(qcount, 0, 1, st);
  if (e == hipSuccess) e = launch_fill_u64(blk, 0, (size_t)(nb > 0 ? nb : 1) * kSatBlkWords, st);
  if (e != hipSuccess) return e;
  if (N >= 2) {
    const int64_t ids = xcd_grouped_ids(nb);
    if (ids > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sat_tile, dim3((unsigned)ids), dim3(256), 0, st, bits, N, W, nb, C, E,
                       blk, (unsigned long long*)qcount, queue, qcap);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (qcap > 0) {
      hipLaunchKernelGGL(k_sat_queue, dim3((unsigned)queue_grid), dim3(256), 0, st, bits, W, C,
                         E, blk, (const unsigned long long*)qcount, queue, qcap);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  hipLaunchKernelGGL(k_sat_reduce, dim3(5), dim3(256), 0, st, blk, nb > 0 ? nb : 1, qcount, out);
  return hipGetLastError();
}

}  // namespace cs
