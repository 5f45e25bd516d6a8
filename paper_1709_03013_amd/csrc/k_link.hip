// k_link.hip -- the O(N^2) linking step (Sec. 2.2): the packed, symmetric,
// zero-diagonal causal matrix from time-sorted coordinates.
//
// 2D flat diamond: order statistics instead of pair tests.  In light-cone
// coordinates the relation is a dominance order: k is in the future of i iff
// u_k > u_i and v_k > v_i, in the past iff u_k < u_i and v_k < v_i.  For a
// block K of 64 labels, sort its u values (and separately its v values)
// together with their labels, and keep the prefix masks pu[c] = labels of the
// c smallest u (pv[c] likewise).  Then word K of row i is
//   past:   pu[#{u_k < u_i}] & pv[#{v_k < v_i}]
//   future: ~pu[#{u_k <= u_i}] & ~pv[#{v_k <= v_i}]   (existing labels only)
// where each count is a binary search of the row's coordinate in the block's
// sorted values: 2 x 7 compares per 64-bit word instead of 2 x 64.  Labels
// are time-sorted, so blocks before the row's own hold only its past, blocks
// after it only its future, and its own block both.  Every compare is the
// same binary64 compare as the definition (strict order, ties unrelated), so
// the words are bit-identical to testing every pair.  k_block_tables builds
// the tables (one wave per block: a bitonic sort across the lanes and a
// prefix OR); k_link2d stages the tables of 8 column blocks in LDS and gives
// each lane one row: it writes 8 consecutive words (64 bytes) of its row per
// row block, looping over 16-row-block tall tiles so the tables are loaded
// once per 1024..4096 rows.
//
// 4D flat diamond and de Sitter slab: pair tests.  Each pair is tested once.
// The matrix is cut into blocks
// of 64 x 64 labels; block (I, K) with I < K (rows of block I, columns of
// block K) is tested as 64 wave-wide compares: the 64 lanes are the columns
// k, the rows i = 64I + r come one at a time as wave-uniform coordinates
// (scalar loads), and each compare yields the lane mask of the columns
// related to row i.  That mask is shifted into every lane's own 32-bit
// accumulator by one carry-in add (acc = acc + acc + carry), so after the 64
// rows lane k holds the 64 relation bits of column k against the rows of
// block I: word I of row k, the lower-triangle word.  An in-register 64x64
// bit transpose (permlane / DPP / swizzle exchanges, one bit-field insert
// per step) turns it into word K of the rows of block I, the upper-triangle
// word.  So a block costs 64 compare steps (the 4D and de Sitter tests in
// binary64) plus 64 carry-in adds and one transpose for 4096 pairs, and
// writes both of its mirror words.  (The batched link uses these pair tests
// for its 2D sets too.)
//
// A workgroup of 4 waves owns a tile of 8 x 8 blocks (512 x 512 labels) of
// the upper triangle (row tile <= column tile); wave w takes the column
// blocks 2w and 2w+1 and runs their compares interleaved.  Upper-triangle
// words are collected in LDS and leave as 64-byte row segments (8 words of
// each of the tile's 512 rows); lower-triangle words stay in the lane that
// owns the row and leave as 64-byte segments too.  Diagonal tiles assemble
// all three kinds (upper, lower, diagonal block) in LDS.  Padding words
// (columns past N up to the row stride) are written as zeros.
//
// Relation (Sec. 1.1, strict timelike separation):
//   2D: u_i < u_k and v_i < v_k for i earlier (off-diagonal blocks: labels
//       are time-sorted, so only that order can hold); both orders inside a
//       diagonal block;
//   4D: dt*dt > (dx*dx + dy*dy) + dz*dz with d* = coordinate of k minus
//       coordinate of i.  Rounding is sign-symmetric, so this equals the
//       test written with the earlier element subtracted; dt*dt > 0 implies
//       dt != 0, so equal times are unrelated.
//   de Sitter slab (Sec. 6.1), rows (w = tan eta, x, y) with (x, y) an
//       unnormalised direction: |d eta| > geodesic angle, which for eta0 <
//       pi/4 reads dot > 0 and |w_i - w_k| * dot > |cross| * (1 + w_i w_k)
//       (tangent of a difference).  Every operand is exactly symmetric in
//       the pair (products commute, a - b = -(b - a)).
// No fused multiply-add anywhere.  An element is never related to itself
// (every test is strict), so the diagonal needs no mask.
#include "cs_internal.h"

#pragma clang fp contract(off)

namespace cs {
namespace {

constexpr int kLT = 8;            // blocks per tile side
constexpr int kRowPad = kLT + 1;  // LDS words per staged row: odd, so 8-byte accesses spread banks

template <int D>
struct Pt {
  double c[D];
};

// Relation of a (the row, wave-uniform) to b (this lane's column) over the
// wave as a 64-bit lane mask.  SYM: either order (a diagonal block);
// otherwise a is the earlier element.  Each compare goes straight to a lane
// mask (no booleans in VGPRs); the masks combine with scalar ANDs.
template <int D, bool SYM>
__device__ __forceinline__ uint64_t related_mask(const Pt<D>& a, const Pt<D>& b) {
  if constexpr (D == 2) {
    const uint64_t fwd = __ballot(a.c[0] < b.c[0]) & __ballot(a.c[1] < b.c[1]);
    if constexpr (!SYM) return fwd;
    return fwd | (__ballot(b.c[0] < a.c[0]) & __ballot(b.c[1] < a.c[1]));
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

// acc * 2 + (this lane's bit of m): one carry-in add shifts the lane mask
// of the newest row into every lane's accumulator.
__device__ __forceinline__ uint32_t shift_in(uint32_t acc, uint64_t m) {
  uint32_t r;
  uint64_t carry_out;
  asm("v_addc_co_u32 %0, %1, %2, %2, %3" : "=v"(r), "=s"(carry_out) : "v"(acc), "s"(m));
  return r;
}

// Lane exchange with lane ^ J inside a 32-bit step of the transpose.
template <int J>
__device__ __forceinline__ uint32_t xchg(uint32_t x) {
  if constexpr (J == 16)
    return (uint32_t)__builtin_amdgcn_ds_swizzle((int)x, (16 << 10) | 0x1F);  // xor 16 in 32
  else if constexpr (J == 8)
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x128, 0xF, 0xF, true);  // row_ror:8
  else if constexpr (J == 4)
    return (uint32_t)__builtin_amdgcn_ds_swizzle((int)x, (4 << 10) | 0x1F);  // xor 4 in 32
  else if constexpr (J == 2)
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x4E, 0xF, 0xF, true);  // quad 2,3,0,1
  else
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xB1, 0xF, 0xF, true);  // quad 1,0,3,2
}

// (keep & x) | (~keep & y) in one instruction.
__device__ __forceinline__ uint32_t bfi(uint32_t keep, uint32_t x, uint32_t y) {
  uint32_t r;
  asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(r) : "v"(keep), "v"(x), "v"(y));
  return r;
}

// Per-lane constants of the 32-bit transpose steps.  Step J pairs lane bit J
// with bit-index bit J: a lane whose bit J is clear keeps its bits whose
// index has bit J clear and takes its partner's such bits moved up by J; a
// lane whose bit J is set keeps the others and takes the partner's moved
// down by J.  J = 16 and 8 move whole bytes (one byte permute of the word
// and its partner's); J = 4, 2, 1 rotate the partner's word (the bits a
// rotate wraps around land where the lane keeps its own) and insert.
struct TConsts {
  uint32_t sel16, sel8;
  uint32_t keep4, rot4, keep2, rot2, keep1, rot1;
};

__device__ __forceinline__ TConsts tconsts(int lane) {
  TConsts t;
  // byte selectors of v_perm (partner's bytes 4-7, own bytes 0-3)
  t.sel16 = (lane & 16) ? 0x03020706u : 0x05040100u;
  t.sel8 = (lane & 8) ? 0x03070105u : 0x06020400u;
  t.keep4 = (lane & 4) ? 0xF0F0F0F0u : 0x0F0F0F0Fu;
  t.rot4 = (lane & 4) ? 4u : 28u;
  t.keep2 = (lane & 2) ? 0xCCCCCCCCu : 0x33333333u;
  t.rot2 = (lane & 2) ? 2u : 30u;
  t.keep1 = (lane & 1) ? 0xAAAAAAAAu : 0x55555555u;
  t.rot1 = (lane & 1) ? 1u : 31u;
  return t;
}

template <int J>
__device__ __forceinline__ uint32_t tbits(uint32_t x, uint32_t keep, uint32_t rot) {
  const uint32_t p = xchg<J>(x);
  return bfi(keep, x, __builtin_amdgcn_alignbit(p, p, rot));
}

// 64x64 bit transpose across the wave: lane k's bit b moves to lane b's
// bit k.  First the two 32x32 off-diagonal quarters trade places (lanes
// 32-63 of the low words with lanes 0-31 of the high words, one permlane
// swap), then the 32x32 transposes run on both halves at once.
__device__ __forceinline__ uint64_t transpose64(uint64_t w, const TConsts& t) {
  const auto q = __builtin_amdgcn_permlane32_swap((uint32_t)w, (uint32_t)(w >> 32), false, false);
  uint32_t lo = q[0], hi = q[1];
  lo = __builtin_amdgcn_perm(xchg<16>(lo), lo, t.sel16);
  hi = __builtin_amdgcn_perm(xchg<16>(hi), hi, t.sel16);
  lo = __builtin_amdgcn_perm(xchg<8>(lo), lo, t.sel8);
  hi = __builtin_amdgcn_perm(xchg<8>(hi), hi, t.sel8);
  lo = tbits<4>(lo, t.keep4, t.rot4);
  hi = tbits<4>(hi, t.keep4, t.rot4);
  lo = tbits<2>(lo, t.keep2, t.rot2);
  hi = tbits<2>(hi, t.keep2, t.rot2);
  lo = tbits<1>(lo, t.keep1, t.rot1);
  hi = tbits<1>(hi, t.keep1, t.rot1);
  return (uint64_t)lo | ((uint64_t)hi << 32);
}

// Coordinates of label i (clamped to the last element; callers mask).
template <int D>
__device__ __forceinline__ Pt<D> point(const double* __restrict__ coords, int64_t N, int64_t i) {
  Pt<D> p;
  const int64_t j = i < N ? i : N - 1;
#pragma unroll
  for (int q = 0; q < D; ++q) p.c[q] = coords[(int64_t)q * N + j];
  return p;
}

// Two column blocks against one earlier row block I (all 64 rows exist):
// lane k gets word I of rows 64K0 + k and 64K1 + k (columns past N are
// cleared by the caller).  Rows arrive in groups of four (scalar loads of
// each coordinate), the next group loaded while the current one is
// compared; a group's eight compare masks are formed before any is shifted
// in, so the compare -> AND -> add chains of different rows overlap.
template <int D>
__device__ __forceinline__ void block_pair(const double* __restrict__ coords, int64_t N, int64_t I,
                                           const Pt<D>& p0, const Pt<D>& p1, uint64_t* w0,
                                           uint64_t* w1) {
  constexpr int G = 4;
  const double* rc[D];
#pragma unroll
  for (int q = 0; q < D; ++q) rc[q] = coords + (int64_t)q * N + I * 64;
  auto load = [&](int r0, Pt<D> (&g)[G]) {
#pragma unroll
    for (int j = 0; j < G; ++j)
#pragma unroll
      for (int q = 0; q < D; ++q) g[j].c[q] = rc[q][r0 - j];
  };
  // One group: the eight compare masks, then the next group's coordinates
  // into the same registers (r_next < 0: none), then the eight carry-in adds
  // while those loads are in flight.
  auto step = [&](Pt<D> (&g)[G], int r_next, uint32_t& a0, uint32_t& a1) {
    uint64_t m0[G], m1[G];
#pragma unroll
    for (int j = 0; j < G; ++j) {
      m0[j] = related_mask<D, false>(g[j], p0);
      m1[j] = related_mask<D, false>(g[j], p1);
    }
    if (r_next >= 0) load(r_next, g);
#pragma unroll
    for (int j = 0; j < G; ++j) {
      a0 = shift_in(a0, m0[j]);
      a1 = shift_in(a1, m1[j]);
    }
  };
  uint32_t h0 = 0, h1 = 0, l0 = 0, l1 = 0;
  Pt<D> cur[G];
  load(63, cur);
#pragma unroll 2
  for (int g = 0; g < 32 / G; ++g)  // rows 63..32: the high words
    step(cur, 63 - G * (g + 1), h0, h1);
#pragma unroll 2
  for (int g = 0; g < 32 / G; ++g)  // rows 31..0: the low words
    step(cur, g + 1 < 32 / G ? 31 - G * (g + 1) : -1, l0, l1);
  *w0 = (uint64_t)l0 | ((uint64_t)h0 << 32);
  *w1 = (uint64_t)l1 | ((uint64_t)h1 << 32);
}

// One column block against row block I <= K: lane k gets word I of row
// 64K + k.  SYM for the diagonal block.  Rows past N contribute no bits.
template <int D, bool SYM>
__device__ __forceinline__ uint64_t block_one(const double* __restrict__ coords, int64_t N, int64_t I,
                                              const Pt<D>& p, uint64_t km) {
  uint32_t h = 0, l = 0;
  const int64_t nrows = N - I * 64;  // rows of block I that exist (>= 1)
  for (int r = 63; r >= 0; --r) {
    const Pt<D> a = point<D>(coords, N, I * 64 + r);
    const uint64_t m = r < nrows ? (related_mask<D, SYM>(a, p) & km) : 0ull;
    if (r >= 32)
      h = shift_in(h, m);
    else
      l = shift_in(l, m);
  }
  return (uint64_t)l | ((uint64_t)h << 32);
}

// Tiles of R row blocks x kLT column blocks (R divides kLT).  Row tile ti
// holds row blocks R*ti .. R*ti+R-1; column tile tk holds column blocks (and
// words) kLT*tk .. kLT*tk+kLT-1.  Only column tiles that reach the diagonal
// or beyond are needed: tk >= floor(R*ti / kLT).
template <int R>
__host__ __device__ inline int64_t first_col_tile(int64_t ti) {
  return (R * ti) / kLT;
}

// Tiles in row tiles 0..T-1: T*nct - sum_{t<T} floor(t/q), q = kLT/R.
template <int R>
__host__ __device__ inline int64_t tiles_before(int64_t T, int64_t nct) {
  constexpr int64_t q = kLT / R;
  const int64_t a = T / q, b = T % q;
  return T * nct - (q * a * (a - 1) / 2 + a * b);
}

template <int R>
__device__ __forceinline__ void tile_of(int64_t id, int64_t nrt, int64_t nct, int64_t* ti,
                                        int64_t* tk) {
  int64_t lo = 0, hi = nrt - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (tiles_before<R>(mid, nct) <= id)
      lo = mid;
    else
      hi = mid - 1;
  }
  *ti = lo;
  *tk = first_col_tile<R>(lo) + (id - tiles_before<R>(lo, nct));
}

// LDS staging of a tile's words (one raw array, views per R):
//  up:  the rows of min(R, 4) row blocks x kLT words of the column tile, row
//       stride kRowPad (odd, so 64 lanes writing one word of 64 rows spread
//       over the banks); flushed every min(R, 4) row blocks;
//  low: the 512 rows of the column tile x R words of the row tile, word w of
//       row r at w ^ ((r >> 1) & (R - 1)).
template <int R>
constexpr int up_words() {
  return (R < 4 ? R : 4) * 64 * kRowPad;
}
template <int R>
constexpr int stage_words() {
  return up_words<R>() + kLT * 64 * R;
}

template <int R>
__device__ __forceinline__ int lpos(int r, int w) {
  return r * R + (w ^ ((r >> 1) & (R - 1)));
}

// The tile (ti, tk) by one 256-thread workgroup.  Wave w owns column blocks
// 2w and 2w+1 of the tile.  For a row block I and a column block K of the
// tile: I < K, the block is tested and gives the lower-triangle words (rows
// of K, word I: low) and, transposed, the upper-triangle words (rows of I,
// word K: up); I == K, the diagonal block gives its own words (up); I > K
// belongs to another tile (as its K < I pair).  Columns past the last
// element up to the row stride are written as zero words (up).  A flush
// skips staged words the tile did not produce (only in tiles that cross
// the diagonal).
template <int D, int R>
__device__ __forceinline__ void link_tile(const double* __restrict__ coords, int64_t N,
                                          uint64_t* __restrict__ bits, int64_t W, int64_t ti,
                                          int64_t tk, uint64_t* st) {
  constexpr int UR = R < 4 ? R : 4;  // row blocks per up flush
  uint64_t* up = st;
  uint64_t* low = st + up_words<R>();
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t NB = (N + 63) >> 6;  // blocks that hold elements
  const int64_t I0 = R * ti, K0 = kLT * tk;
  const bool crosses = K0 < I0 + R;  // some column block at or before some row block
  const TConsts tc = tconsts(lane);

  int kl[2];
  int64_t K[2];
  bool live[2];
  Pt<D> p[2];
  uint64_t km[2], kv[2];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    kl[c] = 2 * wave + c;
    K[c] = K0 + kl[c];
    live[c] = K[c] < NB;
    const int64_t k = K[c] * 64 + lane;
    km[c] = __ballot(k < N);
    kv[c] = k < N ? ~0ull : 0ull;
    p[c] = point<D>(coords, N, live[c] ? k : 0);
  }
  auto put_up = [&](int il, int c, uint64_t w) { up[((il % UR) * 64 + lane) * kRowPad + kl[c]] = w; };
  auto put_low = [&](int il, int c, uint64_t w) { low[lpos<R>(kl[c] * 64 + lane, il)] = w; };

  for (int il = 0; il < R; ++il) {
    const int64_t I = I0 + il;
    if (I < NB) {
      const bool off0 = live[0] && I < K[0], off1 = live[1] && I < K[1];
      if (off0 && off1) {
        uint64_t w0, w1;
        block_pair<D>(coords, N, I, p[0], p[1], &w0, &w1);
        w0 &= kv[0];
        w1 &= kv[1];
        put_low(il, 0, w0);
        put_low(il, 1, w1);
        put_up(il, 0, transpose64(w0, tc));
        put_up(il, 1, transpose64(w1, tc));
      } else {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          if (live[c] && I == K[c]) {
            put_up(il, c, block_one<D, true>(coords, N, I, p[c], km[c]));
          } else if (live[c] && I < K[c]) {
            const uint64_t w = block_one<D, false>(coords, N, I, p[c], km[c]);
            put_low(il, c, w);
            put_up(il, c, transpose64(w, tc));
          }
        }
      }
    }
#pragma unroll
    for (int c = 0; c < 2; ++c)
      if (!live[c] && K[c] < W) put_up(il, c, 0ull);
    if (il % UR == UR - 1) {
      // rows of row blocks I0+il-UR+1 .. I0+il, words K0 .. K0+7, 16 bytes
      // per lane (W is a multiple of 4: a pair never straddles the row end)
      __syncthreads();
      const int64_t b0 = I0 + il - (UR - 1);
      for (int t = threadIdx.x; t < UR * 64 * 4; t += 256) {
        const int r = t >> 2, q = t & 3;
        const int64_t row = b0 * 64 + r, w = K0 + 2 * q;
        if (row >= N || w >= W) continue;
        // words before the row's own block belong to lower-triangle words
        // written elsewhere (only where the tile crosses the diagonal)
        const int64_t first = crosses ? (row >> 6) : 0;
        const uint64_t x = up[r * kRowPad + 2 * q], y = up[r * kRowPad + 2 * q + 1];
        if (w >= first)
          *(uint4*)(bits + row * W + w) =
              make_uint4((uint32_t)x, (uint32_t)(x >> 32), (uint32_t)y, (uint32_t)(y >> 32));
        else if (w + 1 == first)
          bits[row * W + w + 1] = y;
      }
      __syncthreads();
    }
  }
  // low: rows of the column tile, words I0 .. I0+R-1 of the row blocks
  // before them
  __syncthreads();
  constexpr int PW = R >= 2 ? 2 : 1;  // words per lane
  constexpr int LPR = R / PW;         // lanes per row
  for (int t = threadIdx.x; t < kLT * 64 * LPR; t += 256) {
    const int r = t / LPR, q = t % LPR;
    const int64_t row = K0 * 64 + r, w = I0 + PW * q;
    const int64_t rb = row >> 6;
    if (row >= N) continue;
    if constexpr (PW == 2) {
      const uint64_t x = low[lpos<R>(r, PW * q)], y = low[lpos<R>(r, PW * q + 1)];
      if (w + 1 < rb) {
        *(uint4*)(bits + row * W + w) =
            make_uint4((uint32_t)x, (uint32_t)(x >> 32), (uint32_t)y, (uint32_t)(y >> 32));
      } else if (w < rb) {
        bits[row * W + w] = x;
      }
    } else {
      if (w < rb) bits[row * W + w] = low[lpos<R>(r, 0)];
    }
  }
}

template <int D, int R>
__global__ __launch_bounds__(256) void k_link(const double* __restrict__ coords, int64_t N,
                                              uint64_t* __restrict__ bits, int64_t W,
                                              int64_t nrt, int64_t nct) {
  __shared__ uint64_t stage[stage_words<R>()];
  int64_t ti, tk;
  tile_of<R>((int64_t)blockIdx.x, nrt, nct, &ti, &tk);
  link_tile<D, R>(coords, N, bits, W, ti, tk, stage);
}

// Batched: one workgroup per (set, row tile, column tile) item, tiles of
// kBatchR row blocks.  The ensemble's sets are small (N <= 4096): one row
// block per tile wastes the fewest waves on the blocks below the diagonal
// (512-set ensemble: 2.59 ms per batch with 1, 2.98 with 2, 2.88 with 4).
constexpr int kBatchR = 1;

// Both dimensions' tests in one kernel would take 117 VGPRs (4 waves per
// SIMD); asking for 8 waves keeps it at 56 without spilling (512-set
// ensemble 2.065 -> 2.03 ms).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_batch_link(BatchDev b) {
  __shared__ uint64_t stage[stage_words<kBatchR>()];
  int64_t set, ti, tk;
  unpack_item(b.link_items[blockIdx.x], &set, &ti, &tk);
  const BatchSet bs = b.sets[set];
  if (bs.d == 2)
    link_tile<2, kBatchR>(b.coords + bs.coords_off, bs.N, b.bits + bs.bits_off, bs.W, ti, tk, stage);
  else
    link_tile<4, kBatchR>(b.coords + bs.coords_off, bs.N, b.bits + bs.bits_off, bs.W, ti, tk, stage);
}

// ---- 2D by order statistics ------------------------------------------------
// Table of one block of 64 labels (kTabWords words): su[64] and sv[64] (the
// block's u and v values sorted ascending, +inf for labels past N), pu[65]
// and pv[65] (pu[c]: bits of the labels of the c smallest u), then padding.
constexpr int kTabWords = 264;
constexpr int kTabSV = 64, kTabPU = 128, kTabPV = 193;
constexpr int kLink2dKB = 8;  // column blocks (words) per tile

__device__ __forceinline__ double shfl_xor_d(double x, int m) {
  return __longlong_as_double(__shfl_xor((long long)__double_as_longlong(x), m, 64));
}

// One wave per block: each coordinate sorted with its labels across the
// lanes (bitonic, ties by label, so the order is total), then the prefix OR
// of the labels' bits.
__global__ __launch_bounds__(256) void k_block_tables(const double* __restrict__ coords, int64_t N,
                                                      uint64_t* __restrict__ tabs) {
  const int lane = threadIdx.x & 63;
  const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t NB = (N + 63) >> 6;
  if (b >= NB) return;  // whole wave
  const int64_t e = b * 64 + lane;
  uint64_t* t = tabs + b * kTabWords;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    double x = e < N ? coords[(int64_t)q * N + e] : __builtin_inf();
    int idx = lane;
#pragma unroll
    for (int k = 2; k <= 64; k <<= 1)
#pragma unroll
      for (int j = k >> 1; j > 0; j >>= 1) {
        const double ox = shfl_xor_d(x, j);
        const int oi = __shfl_xor(idx, j, 64);
        const bool other_less = ox < x || (ox == x && oi < idx);
        const bool keep_min = ((lane & k) == 0) == ((lane & j) == 0);
        if (keep_min == other_less) {
          x = ox;
          idx = oi;
        }
      }
    uint64_t incl = 1ull << idx;
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) {
      const uint64_t o = __shfl_up(incl, s, 64);
      if (lane >= s) incl |= o;
    }
    t[q * kTabSV + lane] = (uint64_t)__double_as_longlong(x);
    t[(q ? kTabPV : kTabPU) + lane + 1] = incl;
    if (lane == 0) t[q ? kTabPV : kTabPU] = 0ull;
  }
}

// x >= +0: the next double above x, so that p <= x iff p < next_up(x).
__device__ __forceinline__ double next_up(double x) {
  return __longlong_as_double(__double_as_longlong(x) + 1);
}

// Count of the sorted a[0..63] below q: six halvings reach 0..63, one more
// compare decides 64.
__device__ __forceinline__ int count_below(const double* a, double q) {
  int c = 0;
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) c += a[c + s - 1] < q ? s : 0;
  return c + (a[c] < q ? 1 : 0);
}

// Tile: column blocks K0 .. K0+KB-1 (their tables in LDS) x row blocks
// 4*(rt*RB + r) + wave for r < RB; lane = row.  The searches of the KB words
// run level by level so that 2*KB LDS reads are in flight per step.
template <int KB>
__global__ __launch_bounds__(256) void k_link2d(const double* __restrict__ coords, int64_t N,
                                                uint64_t* __restrict__ bits, int64_t W,
                                                const uint64_t* __restrict__ tabs, int64_t nrt,
                                                int RB) {
  __shared__ uint64_t tl[KB * kTabWords];
  const int64_t rt = (int64_t)blockIdx.x % nrt, ct = (int64_t)blockIdx.x / nrt;
  const int64_t K0 = ct * KB;
  const int64_t NB = (N + 63) >> 6;
  for (int q = threadIdx.x; q < KB * kTabWords; q += 256) {
    const int64_t K = K0 + q / kTabWords;
    tl[q] = K < NB ? tabs[K0 * kTabWords + q] : 0ull;
  }
  __syncthreads();
  const double* tld = (const double*)tl;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int rb = 0; rb < RB; ++rb) {
    const int64_t I = (rt * RB + rb) * 4 + wave;
    if (I >= NB) break;  // whole wave; no barrier follows
    const int64_t i = I * 64 + lane;
    const bool live = i < N;
    const double xu = live ? coords[i] : 0.0, xv = live ? coords[N + i] : 0.0;
    const double nu = next_up(xu), nv = next_up(xv);
    // earlier blocks and the row's own: entries below the row; later
    // blocks: entries at or below it
    double qu[KB], qv[KB];
    int cu[KB], cv[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const bool later = K0 + k > I;
      qu[k] = later ? nu : xu;
      qv[k] = later ? nv : xv;
      cu[k] = 0;
      cv[k] = 0;
    }
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1)
#pragma unroll
      for (int k = 0; k < KB; ++k) {
        cu[k] += tld[k * kTabWords + cu[k] + s - 1] < qu[k] ? s : 0;
        cv[k] += tld[k * kTabWords + kTabSV + cv[k] + s - 1] < qv[k] ? s : 0;
      }
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      cu[k] += tld[k * kTabWords + cu[k]] < qu[k] ? 1 : 0;
      cv[k] += tld[k * kTabWords + kTabSV + cv[k]] < qv[k] ? 1 : 0;
    }
    uint64_t w[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const int64_t K = K0 + k;
      const uint64_t a = tl[k * kTabWords + kTabPU + cu[k]], b = tl[k * kTabWords + kTabPV + cv[k]];
      const uint64_t valid =
          K * 64 + 64 <= N ? ~0ull : (K * 64 < N ? ((1ull << (N - K * 64)) - 1ull) : 0ull);
      w[k] = K > I ? (~a & ~b & valid) : (a & b);
    }
    // the row's own block also holds the later elements of that block
    const int64_t kd = I - K0;
    if (kd >= 0 && kd < KB) {
#pragma unroll
      for (int k = 0; k < KB; ++k) {
        if (k != kd) continue;
        const int du = count_below(tld + k * kTabWords, nu);
        const int dv = count_below(tld + k * kTabWords + kTabSV, nv);
        const int64_t K = K0 + k;
        const uint64_t valid = K * 64 + 64 <= N ? ~0ull : ((1ull << (N - K * 64)) - 1ull);
        w[k] |= ~tl[k * kTabWords + kTabPU + du] & ~tl[k * kTabWords + kTabPV + dv] & valid;
      }
    }
    if (live) {
      uint64_t* row = bits + i * W + K0;
#pragma unroll
      for (int k = 0; k < KB; k += 2)
        if (K0 + k < W)
          *(uint4*)(row + k) = make_uint4((uint32_t)w[k], (uint32_t)(w[k] >> 32), (uint32_t)w[k + 1],
                                          (uint32_t)(w[k + 1] >> 32));
    }
  }
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

namespace {
template <int R>
int64_t tile_count(int64_t N, int64_t W) {
  const int64_t nb = (N + 63) / 64;
  return tiles_before<R>((nb + R - 1) / R, (W + kLT - 1) / kLT);
}

template <int D, int R>
hipError_t launch_r(int64_t N, const double* coords, uint64_t* bits, int64_t W, hipStream_t st) {
  const int64_t nb = (N + 63) / 64;
  const int64_t nrt = (nb + R - 1) / R, nct = (W + kLT - 1) / kLT;
  const int64_t tiles = tiles_before<R>(nrt, nct);
  if (tiles > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_link<D, R>), dim3((unsigned)tiles), dim3(256), 0, st, coords, N, bits, W,
                     nrt, nct);
  return hipGetLastError();
}

template <int D>
hipError_t launch_d(int64_t N, const double* coords, uint64_t* bits, int64_t W, hipStream_t st) {
  // the tallest tile that still leaves enough tiles to fill the chip: about
  // 1500 workgroups are resident at once, so at least five rounds of them
  // (4D N = 16384: 0.074 ms with one-row-block tiles against 0.084 ms with
  // the two-row-block tiles a 2048-tile floor chose)
  constexpr int64_t kEnough = 8192;
  if (tile_count<8>(N, W) >= kEnough) return launch_r<D, 8>(N, coords, bits, W, st);
  if (tile_count<4>(N, W) >= kEnough) return launch_r<D, 4>(N, coords, bits, W, st);
  if (tile_count<2>(N, W) >= kEnough) return launch_r<D, 2>(N, coords, bits, W, st);
  return launch_r<D, 1>(N, coords, bits, W, st);
}
}  // namespace

int64_t batch_link_tiles(int64_t N, int64_t W, int64_t* nrt, int64_t* nct) {
  const int64_t nb = (N + 63) / 64;
  *nrt = (nb + kBatchR - 1) / kBatchR;
  *nct = (W + kLT - 1) / kLT;
  return tiles_before<kBatchR>(*nrt, *nct);
}

int64_t batch_link_first_col(int64_t ti) { return first_col_tile<kBatchR>(ti); }

size_t link_workspace_bytes(int d, int64_t N) {
  return d == 2 && N > 0 ? (size_t)((N + 63) / 64) * kTabWords * 8 : 0;
}

hipError_t launch_link(int d, int64_t N, const double* coords, uint64_t* bits,
                       int64_t W, void* work, hipStream_t st) {
  if (N <= 0) return hipSuccess;
  if (d == 2) {
    if (!work) return hipErrorInvalidValue;
    uint64_t* tabs = (uint64_t*)work;
    const int64_t NB = (N + 63) / 64;
    hipLaunchKernelGGL(k_block_tables, dim3((unsigned)((NB + 3) / 4)), dim3(256), 0, st, coords, N, tabs);
    // row blocks per tile: the tallest (up to 16 x 4) that leaves at least
    // 2048 tiles, so the tables are loaded once per many rows
    constexpr int KB = kLink2dKB;
    const int64_t nct = (W + KB - 1) / KB;
    int RB = 16;
    while (RB > 1 && ((NB + 4 * RB - 1) / (4 * RB)) * nct < 2048) RB >>= 1;
    const int64_t nrt = (NB + 4 * RB - 1) / (4 * RB);
    if (nrt * nct > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_link2d<KB>), dim3((unsigned)(nrt * nct)), dim3(256), 0, st, coords, N, bits, W,
                       (const uint64_t*)tabs, nrt, RB);
    return hipGetLastError();
  }
  if (d == kLinkDeSitter) return launch_d<3>(N, coords, bits, W, st);
  return launch_d<4>(N, coords, bits, W, st);
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
