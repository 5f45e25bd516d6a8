// k_link.hip -- the O(N^2) linking step (Sec. 2.2): the packed, symmetric,
// zero-diagonal causal matrix from time-sorted coordinates.
//
// gfx950 design: a wave's 64 lanes are 64 consecutive columns k of a 64-bit
// word (four words per pass: columns k, k+64, k+128, k+192 per lane); for
// each row i (wave-uniform, coordinates broadcast from LDS) the relation
// tests produce each word directly as the wave's compare mask, written into
// lane i%64 with v_writelane (one M0 lane select per row for the four
// words).  After 64 rows every lane holds its row's words of a 64x64-word
// tile, which is staged in LDS and stored row by row with fully coalesced
// 512-byte rows.
//
// Relation (Sec. 1.1, strict timelike separation), for either order of the
// pair, so the symmetric matrix needs no index test:
//   2D: (u_i < u_k and v_i < v_k) or (u_k < u_i and v_k < v_i);
//   4D: dt*dt > (dx*dx + dy*dy) + dz*dz with d* = coordinate of k minus
//       coordinate of i.  Rounding is sign-symmetric, so this equals the
//       test written with the earlier element subtracted; dt*dt > 0 implies
//       dt != 0, so equal times are unrelated.
//   de Sitter slab (Sec. 6.1), rows (w = tan eta, x, y) with (x, y) an
//       unnormalised direction: |d eta| > geodesic angle, which for eta0 <
//       pi/4 reads dot > 0 and |w_i - w_k| * dot > |cross| * (1 + w_i w_k)
//       (tangent of a difference).  Every operand is exactly symmetric in the
//       pair (products commute, a - b = -(b - a)).
// No fused multiply-add anywhere.
#include <cstdlib>

#include "cs_internal.h"

#pragma clang fp contract(off)

namespace cs {
namespace {

template <int D>
struct Pt {
  double c[D];
};

// Relation of a (the row, wave-uniform) to b (this lane's column) over the
// wave, as a 64-bit lane mask (Sec. 1.1, strict).  DIR: 0 = either order
// (the diagonal 64x64 block), 1 = a before b (columns after the rows), 2 = b
// before a.  Each comparison goes straight to a lane mask (no booleans in
// VGPRs) and the masks are combined with scalar ANDs.
template <int D, int DIR>
__device__ __forceinline__ uint64_t related_mask(const Pt<D>& a, const Pt<D>& b) {
  if constexpr (D == 2) {
    const uint64_t fwd = __ballot(a.c[0] < b.c[0]) & __ballot(a.c[1] < b.c[1]);
    if constexpr (DIR == 1) return fwd;
    const uint64_t bwd = __ballot(b.c[0] < a.c[0]) & __ballot(b.c[1] < a.c[1]);
    if constexpr (DIR == 2) return bwd;
    return fwd | bwd;
  } else if constexpr (D == 3) {
    const double dot = a.c[1] * b.c[1] + a.c[2] * b.c[2];
    const double cr = fabs(a.c[1] * b.c[2] - a.c[2] * b.c[1]);
    const double dw = fabs(a.c[0] - b.c[0]);
    const double bb = 1.0 + a.c[0] * b.c[0];
    return __ballot(dot > 0.0) & __ballot(dw * dot > cr * bb);
  } else {
    const double dt = b.c[0] - a.c[0];
    const double dx = b.c[1] - a.c[1];
    const double dy = b.c[2] - a.c[2];
    const double dz = b.c[3] - a.c[3];
    const double tt = dt * dt;
    const double xx = dx * dx, yy = dy * dy, zz = dz * dz;
    return __ballot(tt > (xx + yy) + zz);
  }
}

// 64 relation words of one column word: lane r ends with word (i0 + r, w).
// The row's coordinates are LDS broadcasts; each row's word is the wave's
// compare mask, written into lane r with v_writelane.
template <int D, int DIR, bool PARTIAL>
__device__ __forceinline__ uint64_t link_word(const double (*rowc)[64], const Pt<D>& pk,
                                              uint64_t kmask) {
  int lo = 0, hi = 0;
#pragma unroll 8
  for (int r = 0; r < 64; ++r) {
    Pt<D> pi;
#pragma unroll
    for (int q = 0; q < D; ++q) pi.c[q] = rowc[q][r];
    const uint64_t rel = related_mask<D, DIR>(pi, pk);
    const uint64_t m = PARTIAL ? (kmask & rel) : rel;
    const int mlo = (int)(uint32_t)m, mhi = (int)(uint32_t)(m >> 32);
    // the lane select goes through M0 (one SGPR operand per VOP3 on gfx9);
    // hipcc warns that M0 is reserved: the link kernels' own code keeps no
    // value in M0 (their only M0 writes are these statements)
    asm("s_mov_b32 m0, %4\n\tv_writelane_b32 %0, %2, m0\n\tv_writelane_b32 %1, %3, m0"
        : "+v"(lo), "+v"(hi)
        : "s"(mlo), "s"(mhi), "s"(r)
        : "m0");
  }
  return (uint64_t)(uint32_t)lo | ((uint64_t)(uint32_t)hi << 32);
}

// The same for two column words at once (this lane's columns k and k + 64):
// one LDS broadcast and one lane select per row serve both.
template <int D, int DIR, bool PARTIAL>
__device__ __forceinline__ void link_word2(const double (*rowc)[64], const Pt<D>& pk0,
                                           const Pt<D>& pk1, uint64_t kmask0, uint64_t kmask1,
                                           uint64_t* my0, uint64_t* my1) {
  int lo0 = 0, hi0 = 0, lo1 = 0, hi1 = 0;
#pragma unroll 4
  for (int r = 0; r < 64; ++r) {
    Pt<D> pi;
#pragma unroll
    for (int q = 0; q < D; ++q) pi.c[q] = rowc[q][r];
    const uint64_t r0 = related_mask<D, DIR>(pi, pk0), r1 = related_mask<D, DIR>(pi, pk1);
    const uint64_t m0 = PARTIAL ? (kmask0 & r0) : r0;
    const uint64_t m1 = PARTIAL ? (kmask1 & r1) : r1;
    asm("s_mov_b32 m0, %8\n\tv_writelane_b32 %0, %4, m0\n\tv_writelane_b32 %1, %5, m0\n\t"
        "v_writelane_b32 %2, %6, m0\n\tv_writelane_b32 %3, %7, m0"
        : "+v"(lo0), "+v"(hi0), "+v"(lo1), "+v"(hi1)
        : "s"((int)(uint32_t)m0), "s"((int)(uint32_t)(m0 >> 32)), "s"((int)(uint32_t)m1),
          "s"((int)(uint32_t)(m1 >> 32)), "s"(r)
        : "m0");
  }
  *my0 = (uint64_t)(uint32_t)lo0 | ((uint64_t)(uint32_t)hi0 << 32);
  *my1 = (uint64_t)(uint32_t)lo1 | ((uint64_t)(uint32_t)hi1 << 32);
}

// Four column words at once (columns k + 64u, u = 0..3).
template <int D, int DIR, bool PARTIAL>
__device__ __forceinline__ void link_word4(const double (*rowc)[64], const Pt<D> (&pk)[4],
                                           const uint64_t (&km)[4], uint64_t (&my)[4]) {
  int lo0 = 0, hi0 = 0, lo1 = 0, hi1 = 0, lo2 = 0, hi2 = 0, lo3 = 0, hi3 = 0;
#pragma unroll 2
  for (int r = 0; r < 64; ++r) {
    Pt<D> pi;
#pragma unroll
    for (int q = 0; q < D; ++q) pi.c[q] = rowc[q][r];
    uint64_t m[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint64_t rel = related_mask<D, DIR>(pi, pk[u]);
      m[u] = PARTIAL ? (km[u] & rel) : rel;
    }
    asm("s_mov_b32 m0, %16\n\t"
        "v_writelane_b32 %0, %8, m0\n\tv_writelane_b32 %1, %9, m0\n\t"
        "v_writelane_b32 %2, %10, m0\n\tv_writelane_b32 %3, %11, m0\n\t"
        "v_writelane_b32 %4, %12, m0\n\tv_writelane_b32 %5, %13, m0\n\t"
        "v_writelane_b32 %6, %14, m0\n\tv_writelane_b32 %7, %15, m0"
        : "+v"(lo0), "+v"(hi0), "+v"(lo1), "+v"(hi1), "+v"(lo2), "+v"(hi2), "+v"(lo3), "+v"(hi3)
        : "s"((int)(uint32_t)m[0]), "s"((int)(uint32_t)(m[0] >> 32)), "s"((int)(uint32_t)m[1]),
          "s"((int)(uint32_t)(m[1] >> 32)), "s"((int)(uint32_t)m[2]), "s"((int)(uint32_t)(m[2] >> 32)),
          "s"((int)(uint32_t)m[3]), "s"((int)(uint32_t)(m[3] >> 32)), "s"(r)
        : "m0");
  }
  my[0] = (uint64_t)(uint32_t)lo0 | ((uint64_t)(uint32_t)hi0 << 32);
  my[1] = (uint64_t)(uint32_t)lo1 | ((uint64_t)(uint32_t)hi1 << 32);
  my[2] = (uint64_t)(uint32_t)lo2 | ((uint64_t)(uint32_t)hi2 << 32);
  my[3] = (uint64_t)(uint32_t)lo3 | ((uint64_t)(uint32_t)hi3 << 32);
}

// One 64-row x 64-word tile of the matrix, rows i0.., words w0.. (256 threads).
// The 64 rows' coordinates are staged in LDS and read as broadcasts; each
// wave builds 16 words, one column word (64 columns, one per lane) at a time,
// and the tile leaves through LDS as coalesced 512-byte row segments.  Off
// the diagonal block only one order of each pair can hold (labels are
// time-sorted), so only that direction is tested.
template <int D, int NW = 1>
__device__ __forceinline__ void link_tile(const double* __restrict__ coords, int64_t N,
                                          uint64_t* __restrict__ bits, int64_t W,
                                          int64_t i0, int64_t w0,
                                          uint64_t (*tile)[65], double (*rowc)[64]) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  if (threadIdx.x < 64) {
    const int64_t i = i0 + lane;
#pragma unroll
    for (int q = 0; q < D; ++q) rowc[q][lane] = i < N ? coords[(int64_t)q * N + i] : 0.0;
  }
  __syncthreads();
  if constexpr (NW == 4) {
    for (int wl = 0; wl < 16; wl += 4) {
      const int wloc = wave * 16 + wl;
      const int64_t w = w0 + wloc;  // words w .. w + 3
      uint64_t my[4] = {0, 0, 0, 0};
      if (w < W) {  // W is a multiple of 4 and w of 4, so w + 3 < W too
        Pt<D> pk[4];
        uint64_t km[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int64_t k = (w + u) * 64 + lane;
          km[u] = __ballot(k < N);
#pragma unroll
          for (int q = 0; q < D; ++q) pk[u].c[q] = coords[(int64_t)q * N + (k < N ? k : 0)];
        }
        if (km[3] != ~0ull)  // a column past N: the last words only
          link_word4<D, 0, true>(rowc, pk, km, my);
        else if (w * 64 >= i0 + 64)
          link_word4<D, 1, false>(rowc, pk, km, my);
        else if (w * 64 + 256 <= i0)
          link_word4<D, 2, false>(rowc, pk, km, my);
        else
          link_word4<D, 0, false>(rowc, pk, km, my);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) tile[lane][wloc + u] = my[u];
    }
  } else if constexpr (NW == 2) {
    for (int wl = 0; wl < 16; wl += 2) {
      const int wloc = wave * 16 + wl;
      const int64_t w = w0 + wloc;  // words w and w + 1
      uint64_t my0 = 0, my1 = 0;
      if (w < W) {  // W is a multiple of 4, so w + 1 < W too
        const int64_t k0 = w * 64 + lane, k1 = k0 + 64;
        const uint64_t km0 = __ballot(k0 < N), km1 = __ballot(k1 < N);
        Pt<D> p0, p1;
#pragma unroll
        for (int q = 0; q < D; ++q) {
          p0.c[q] = coords[(int64_t)q * N + (k0 < N ? k0 : 0)];
          p1.c[q] = coords[(int64_t)q * N + (k1 < N ? k1 : 0)];
        }
        if (km1 != ~0ull)  // a column past N: the last words only
          link_word2<D, 0, true>(rowc, p0, p1, km0, km1, &my0, &my1);
        else if (w * 64 >= i0 + 64)
          link_word2<D, 1, false>(rowc, p0, p1, km0, km1, &my0, &my1);
        else if (w * 64 + 128 <= i0)
          link_word2<D, 2, false>(rowc, p0, p1, km0, km1, &my0, &my1);
        else
          link_word2<D, 0, false>(rowc, p0, p1, km0, km1, &my0, &my1);
      }
      tile[lane][wloc] = my0;
      tile[lane][wloc + 1] = my1;
    }
  } else {
    for (int wl = 0; wl < 16; ++wl) {
      const int wloc = wave * 16 + wl;
      const int64_t w = w0 + wloc;
      uint64_t my = 0;
      if (w < W) {
        const int64_t k = w * 64 + lane;
        const bool kval = k < N;
        const uint64_t kmask = __ballot(kval);
        const int64_t kk = kval ? k : 0;
        Pt<D> pk;
#pragma unroll
        for (int q = 0; q < D; ++q) pk.c[q] = coords[(int64_t)q * N + kk];
        if (kmask != ~0ull)  // a column past N: the last word only
          my = link_word<D, 0, true>(rowc, pk, kmask);
        else if (w * 64 >= i0 + 64)
          my = link_word<D, 1, false>(rowc, pk, kmask);
        else if (w * 64 + 64 <= i0)
          my = link_word<D, 2, false>(rowc, pk, kmask);
        else
          my = link_word<D, 0, false>(rowc, pk, kmask);
      }
      tile[lane][wloc] = my;
    }
  }
  __syncthreads();
  for (int p = 0; p < 16; ++p) {
    const int r = p * 4 + wave;
    const int64_t i = i0 + r;
    const int64_t w = w0 + lane;
    if (i < N && w < W) bits[i * W + w] = tile[r][lane];
  }
}

template <int D, int NW>
__global__ __launch_bounds__(256) void k_link(const double* __restrict__ coords,
                                              int64_t N,
                                              uint64_t* __restrict__ bits,
                                              int64_t W) {
  __shared__ uint64_t tile[64][65];
  __shared__ double rowc[D][64];
  link_tile<D, NW>(coords, N, bits, W, (int64_t)blockIdx.y * 64, (int64_t)blockIdx.x * 64, tile, rowc);
}

// Batched: one workgroup per (set, 64-row tile, 64-word tile) item.
__global__ __launch_bounds__(256) void k_batch_link(BatchDev b) {
  __shared__ uint64_t tile[64][65];
  __shared__ double rowc[4][64];
  int64_t set, ti, tw;
  unpack_item(b.link_items[blockIdx.x], &set, &ti, &tw);
  const BatchSet bs = b.sets[set];
  if (bs.d == 2)
    link_tile<2, 4>(b.coords + bs.coords_off, bs.N, b.bits + bs.bits_off, bs.W, ti * 64, tw * 64,
                    tile, rowc);
  else
    link_tile<4, 4>(b.coords + bs.coords_off, bs.N, b.bits + bs.bits_off, bs.W, ti * 64, tw * 64,
                    tile, rowc);
}

__global__ __launch_bounds__(256) void k_fill_u64(uint64_t* __restrict__ p,
                                                  uint64_t v, size_t n) {
  size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * 256;
  for (; e < n; e += stride) p[e] = v;
}

// One thread per word (i, w): padding bits zero, diagonal bit zero, and every
// set bit k has its mirror bit (k, i) set.
__global__ __launch_bounds__(256) void k_validate(const uint64_t* __restrict__ bits,
                                                  int64_t N, int64_t W,
                                                  uint32_t* __restrict__ bad) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= N * W) return;
  const int64_t i = e / W, w = e % W;
  uint64_t x = bits[e];
  uint32_t fault = 0;
  const int64_t base = w * 64;
  if (base + 64 > N) {
    const uint64_t keep = base >= N ? 0ull : ((1ull << (N - base)) - 1);
    if (x & ~keep) fault = 1;
    x &= keep;
  }
  if ((i >> 6) == w && ((x >> (i & 63)) & 1ull)) fault = 1;
  while (x) {
    const int b = __ffsll((unsigned long long)x) - 1;
    x &= x - 1;
    const int64_t k = base + b;
    if (!((bits[k * W + (i >> 6)] >> (i & 63)) & 1ull)) fault = 1;
  }
  if (fault) atomicOr(bad, 1u);
}

}  // namespace

hipError_t launch_link(int d, int64_t N, const double* coords, uint64_t* bits,
                       int64_t W, hipStream_t st) {
  if (N <= 0) return hipSuccess;
  dim3 grid((unsigned)((W + 63) / 64), (unsigned)((N + 63) / 64));
  // Column words per pass over the 64 rows: 4 by default (2D N=2^17: 1 word
  // 3.7 ms, 2 words 2.3 ms); CS_LINK_VARIANT = 1 or 2 selects 1 or 2 for timing.
  const char* ev = getenv("CS_LINK_VARIANT");
  const int nw = ev && ev[0] == '1' ? 1 : (ev && ev[0] == '2' ? 2 : 4);
  if (nw == 4) {
    if (d == 2)
      hipLaunchKernelGGL((k_link<2, 4>), grid, dim3(256), 0, st, coords, N, bits, W);
    else if (d == kLinkDeSitter)
      hipLaunchKernelGGL((k_link<3, 4>), grid, dim3(256), 0, st, coords, N, bits, W);
    else
      hipLaunchKernelGGL((k_link<4, 4>), grid, dim3(256), 0, st, coords, N, bits, W);
  } else if (nw == 2) {
    if (d == 2)
      hipLaunchKernelGGL((k_link<2, 2>), grid, dim3(256), 0, st, coords, N, bits, W);
    else if (d == kLinkDeSitter)
      hipLaunchKernelGGL((k_link<3, 2>), grid, dim3(256), 0, st, coords, N, bits, W);
    else
      hipLaunchKernelGGL((k_link<4, 2>), grid, dim3(256), 0, st, coords, N, bits, W);
  } else {
    if (d == 2)
      hipLaunchKernelGGL((k_link<2, 1>), grid, dim3(256), 0, st, coords, N, bits, W);
    else if (d == kLinkDeSitter)
      hipLaunchKernelGGL((k_link<3, 1>), grid, dim3(256), 0, st, coords, N, bits, W);
    else
      hipLaunchKernelGGL((k_link<4, 1>), grid, dim3(256), 0, st, coords, N, bits, W);
  }
  return hipGetLastError();
}

hipError_t launch_batch_link(const BatchDev& b, hipStream_t st) {
  if (b.n_link <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_link, dim3((unsigned)b.n_link), dim3(256), 0, st, b);
  return hipGetLastError();
}

hipError_t launch_fill_u64(uint64_t* p, uint64_t v, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  size_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)blocks), dim3(256), 0, st, p, v, n);
  return hipGetLastError();
}

hipError_t launch_validate(const uint64_t* bits, int64_t N, int64_t W,
                           uint32_t* bad_dev, hipStream_t st) {
  if (N <= 0) return hipSuccess;
  const int64_t n = N * W;
  hipLaunchKernelGGL(k_validate, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     st, bits, N, W, bad_dev);
  return hipGetLastError();
}

}  // namespace cs
