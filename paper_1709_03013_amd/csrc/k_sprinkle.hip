// k_sprinkle.hip -- sprinkling into flat causal diamonds and the time sort.
//
// Sec. 2.1 (coordinates drawn i.i.d. from the normalized volume form, in
// parallel) and Sec. 2.2 (labels sorted by time so that the order is
// topological).  Random numbers: Philox4x64-10 (Salmon et al., SC'11), one
// block of four 64-bit words per element (2D) or candidate (4D), counter
// (c,0,0,0), key (seed, 1) for 2D and (seed, 2) for 4D.
//
// 2D: u = (r0>>11) 2^-53, v = (r1>>11) 2^-53; with a = r0>>11, b = r1>>11 the
//     time (u+v)/2 = (a+b) 2^-54 is exact, so the sort key is (a+b, a, c).
// 4D: candidate c: t = dbl(r0), x,y,z = dbl(r1..r3) - 1/2, accepted iff
//     (x*x + y*y) + z*z < m*m with m = min(t, 1-t) (binary64, no fused
//     multiply-add).  The first N accepted in candidate order are the
//     elements, sorted by (r0>>11, acceptance rank).
//
// (1+1) de Sitter slab (Sec. 6.1, Eq. 9): the volume element sec^2(eta)
//     deta dtheta is dw dtheta with w = tan(eta), so elements are uniform in
//     w on [-w0, w0] (w0 = tan(eta0)) and in angle.  Element c, attempt a =
//     0..63, block at counter (c, a, 0, 0), key (seed, 5): w = (2 dbl(r0) - 1)
//     w0; the direction (x, y) = 2 dbl(r1..r2) - 1 is accepted iff 0 < x*x +
//     y*y < 1 (after 64 rejections: (1, 0)).  Sorted by (w, c).
//
// Sort: each workgroup bitonic-sorts a tile of 2048 records in LDS; every
// record then finds its global rank as its rank in its own tile plus the
// number of smaller records in every other tile (binary search), and
// scatters its coordinates there.  Keys are unique, so ranks are a
// permutation.
#include "cs_internal.h"

#pragma clang fp contract(off)

namespace cs {
namespace {

constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kM1 = 0xCA5A826395121157ull;
constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kW1 = 0xBB67AE8584CAA73Bull;

__device__ __forceinline__ void philox10(uint64_t c[4], uint64_t k0,
                                         uint64_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += kW0;
      k1 += kW1;
    }
    const uint64_t lo0 = kM0 * c[0], hi0 = __umul64hi(kM0, c[0]);
    const uint64_t lo1 = kM1 * c[2], hi1 = __umul64hi(kM1, c[2]);
    const uint64_t n0 = hi1 ^ c[1] ^ k0;
    const uint64_t n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

__device__ __forceinline__ double unit53(uint64_t r) {
  return (double)(r >> 11) * 0x1.0p-53;
}

// 4D candidate test; returns the coordinates and the integer time key.
__device__ __forceinline__ bool candidate4d(uint64_t c, uint64_t seed,
                                            double xyz[4], uint64_t* kt) {
  uint64_t r[4] = {c, 0, 0, 0};
  philox10(r, seed, 2);
  const double t = unit53(r[0]);
  const double x = unit53(r[1]) - 0.5;
  const double y = unit53(r[2]) - 0.5;
  const double z = unit53(r[3]) - 0.5;
  const double omt = 1.0 - t;
  const double m = t < omt ? t : omt;
  const double xx = x * x, yy = y * y, zz = z * z;
  const double rho2 = (xx + yy) + zz;
  const double mm = m * m;
  xyz[0] = t;
  xyz[1] = x;
  xyz[2] = y;
  xyz[3] = z;
  *kt = r[0] >> 11;
  return rho2 < mm;
}

__global__ __launch_bounds__(256) void k_keys2d(int64_t N, uint64_t seed,
                                                SortRec* __restrict__ recs) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= N) return;
  uint64_t r[4] = {(uint64_t)c, 0, 0, 0};
  philox10(r, seed, 1);
  const uint64_t a = r[0] >> 11, b = r[1] >> 11;
  SortRec s;
  s.k1 = a + b;
  s.k2 = a;
  s.idx = (uint64_t)c;
  recs[c] = s;
}

// Order-preserving map of a binary64 to uint64 (w is never -0: (2u - 1) is
// +0 when zero and w0 > 0).
__device__ __forceinline__ uint64_t order_bits(double w) {
  const uint64_t b = (uint64_t)__double_as_longlong(w);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__global__ __launch_bounds__(256) void k_keys_desitter(int64_t N, uint64_t seed, double w0,
                                                       SortRec* __restrict__ recs,
                                                       double* __restrict__ raw) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= N) return;
  double w = 0.0, x = 1.0, y = 0.0;
  for (uint64_t a = 0; a < 64; ++a) {
    uint64_t r[4] = {(uint64_t)c, a, 0, 0};
    philox10(r, seed, 5);
    w = (2.0 * unit53(r[0]) - 1.0) * w0;
    const double xc = 2.0 * unit53(r[1]) - 1.0;
    const double yc = 2.0 * unit53(r[2]) - 1.0;
    const double rr = xc * xc + yc * yc;
    if (rr > 0.0 && rr < 1.0) {
      x = xc;
      y = yc;
      break;
    }
  }
  SortRec s;
  s.k1 = order_bits(w);
  s.k2 = (uint64_t)c;
  s.idx = (uint64_t)c;
  recs[c] = s;
  raw[c] = w;
  raw[N + c] = x;
  raw[2 * N + c] = y;
}

__global__ __launch_bounds__(256) void k_count4d(int64_t ncand, uint64_t seed,
                                                 uint32_t* __restrict__ blkcnt) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double xyz[4];
  uint64_t kt;
  const bool acc = c < ncand && candidate4d((uint64_t)c, seed, xyz, &kt);
  const int n = __syncthreads_count(acc);
  if (threadIdx.x == 0) blkcnt[blockIdx.x] = (uint32_t)n;
}

// Exclusive scan of nblk counts in one workgroup of 1024 threads; also the
// total (number of accepted candidates).
__global__ __launch_bounds__(1024) void k_scan_counts(
    const uint32_t* __restrict__ blkcnt, int64_t nblk,
    uint64_t* __restrict__ offs, uint64_t* __restrict__ total) {
  __shared__ uint64_t part[1024];
  const int tid = threadIdx.x;
  const int64_t per = (nblk + 1023) / 1024;
  const int64_t lo = tid * per;
  const int64_t hi = lo + per < nblk ? lo + per : nblk;
  uint64_t s = 0;
  for (int64_t b = lo; b < hi; ++b) s += blkcnt[b];
  part[tid] = s;
  __syncthreads();
  // Hillis-Steele inclusive scan over 1024 partial sums.
  for (int d = 1; d < 1024; d <<= 1) {
    const uint64_t v = tid >= d ? part[tid - d] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  uint64_t run = part[tid] - s;  // exclusive prefix of this thread's chunk
  for (int64_t b = lo; b < hi; ++b) {
    offs[b] = run;
    run += blkcnt[b];
  }
  if (tid == 1023) *total = part[1023];
}

__global__ __launch_bounds__(256) void k_compact4d(
    int64_t ncand, uint64_t seed, const uint64_t* __restrict__ offs, int64_t N,
    SortRec* __restrict__ recs, double* __restrict__ raw) {
  __shared__ uint32_t wcnt[4];
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double xyz[4];
  uint64_t kt = 0;
  const bool acc = c < ncand && candidate4d((uint64_t)c, seed, xyz, &kt);
  const uint64_t bal = __ballot(acc);
  const uint32_t below = __builtin_amdgcn_mbcnt_hi(
      (uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
  if (lane == 0) wcnt[wave] = (uint32_t)__popcll(bal);
  __syncthreads();
  uint32_t woff = 0;
  for (int q = 0; q < wave; ++q) woff += wcnt[q];
  const int64_t e = (int64_t)(offs[blockIdx.x] + woff + below);
  if (acc && e < N) {
    SortRec s;
    s.k1 = kt;
    s.k2 = 0;
    s.idx = (uint64_t)e;
    recs[e] = s;
    raw[e] = xyz[0];
    raw[N + e] = xyz[1];
    raw[2 * N + e] = xyz[2];
    raw[3 * N + e] = xyz[3];
  }
}

// Lexicographic (k1, k2, idx), without branches: five 64-bit compares whose
// lane masks combine with scalar logic, so a compare-exchange never splits
// the wave.
__device__ __forceinline__ bool rec_less(const SortRec& a, const SortRec& b) {
  const bool lt1 = a.k1 < b.k1, eq1 = a.k1 == b.k1;
  const bool lt2 = a.k2 < b.k2, eq2 = a.k2 == b.k2;
  const bool lt3 = a.idx < b.idx;
  return lt1 | (eq1 & (lt2 | (eq2 & lt3)));
}

// One record of lane ^ m of the wave.
__device__ __forceinline__ SortRec shfl_rec(const SortRec& r, int m) {
  SortRec o;
  o.k1 = (uint64_t)__shfl_xor((long long)r.k1, m, 64);
  o.k2 = (uint64_t)__shfl_xor((long long)r.k2, m, 64);
  o.idx = (uint64_t)__shfl_xor((long long)r.idx, m, 64);
  return o;
}

// c ? b : a, field by field (selects, no branch).
__device__ __forceinline__ SortRec sel(bool c, const SortRec& a, const SortRec& b) {
  SortRec r;
  r.k1 = c ? b.k1 : a.k1;
  r.k2 = c ? b.k2 : a.k2;
  r.idx = c ? b.idx : a.idx;
  return r;
}

// The smaller (lo) or larger of a and b.
__device__ __forceinline__ SortRec pick(const SortRec& a, const SortRec& b, bool lo) {
  return sel(rec_less(b, a) == lo, a, b);
}

// Bitonic sort of n <= kSortTile records at base by 1024 threads, over the
// smallest power of two P >= n (padded with records above every key).
// Thread t holds positions 2t and 2t+1 in registers.  A compare-exchange
// step at distance j pairs position p with p ^ j: j = 1 stays inside the
// thread, 2 <= j <= 64 pairs lanes t and t ^ j/2 of the same wave (lane
// shuffles, no barrier), and only j >= 128 goes through LDS (10 of the 66
// steps of a full tile).  Position p keeps the smaller record iff it is the
// lower of its pair exactly when its block of size k is ascending.
__device__ __forceinline__ void tile_sort_body(SortRec* __restrict__ base, int64_t n,
                                               SortRec* s) {
  const int t = threadIdx.x;
  int P = 2;
  while (P < n) P <<= 1;
  SortRec pad;
  pad.k1 = ~0ull;
  pad.k2 = ~0ull;
  pad.idx = ~0ull;
  const int p0 = 2 * t;
  SortRec r0 = p0 < n ? base[p0] : pad;
  SortRec r1 = p0 + 1 < n ? base[p0 + 1] : pad;
  for (int k = 2; k <= P; k <<= 1) {
    const bool up = (p0 & k) == 0;
    for (int j = k >> 1; j > 0; j >>= 1) {
      if (j == 1) {
        // positions p0 (lower) and p0 + 1
        const bool sw = rec_less(r1, r0) == up;
        const SortRec x = r0;
        r0 = sel(sw, r0, r1);
        r1 = sel(sw, r1, x);
      } else {
        const bool lo = ((p0 & j) == 0) == up;
        SortRec o0, o1;
        if (j <= 64) {
          o0 = shfl_rec(r0, j >> 1);
          o1 = shfl_rec(r1, j >> 1);
        } else {
          s[p0] = r0;
          s[p0 + 1] = r1;
          __syncthreads();
          o0 = s[p0 ^ j];
          o1 = s[(p0 + 1) ^ j];
          __syncthreads();  // before the next step writes s
        }
        r0 = pick(r0, o0, lo);
        r1 = pick(r1, o1, lo);
      }
    }
  }
  if (p0 < n) base[p0] = r0;
  if (p0 + 1 < n) base[p0 + 1] = r1;
}

__global__ __launch_bounds__(1024) void k_tile_sort(SortRec* __restrict__ recs,
                                                    int64_t N) {
  __shared__ SortRec s[kSortTile];
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  const int64_t n = N - base < kSortTile ? N - base : kSortTile;
  tile_sort_body(recs + base, n, s);
}

// Final position of record e of a set: its rank in its own sorted tile plus
// the number of smaller records in every other tile; scatter its
// coordinates there.
template <int D>
__device__ __forceinline__ void rank_scatter_one(const SortRec* __restrict__ recs,
                                                 int64_t N, const double* __restrict__ raw,
                                                 double* __restrict__ coords,
                                                 int64_t* __restrict__ orig, int64_t e) {
  const SortRec my = recs[e];
  if (my.idx >= (uint64_t)N) return;  // unfilled record (too few 4D draws)
  const int64_t mytile = e / kSortTile;
  int64_t rank = e - mytile * kSortTile;
  const int64_t ntiles = (N + kSortTile - 1) / kSortTile;
  for (int64_t u = 0; u < ntiles; ++u) {
    if (u == mytile) continue;
    const int64_t lo = u * kSortTile;
    int64_t len = N - lo < kSortTile ? N - lo : kSortTile;
    // number of records in tile u that are smaller than mine
    int64_t a = 0, b = len;
    while (a < b) {
      const int64_t mid = (a + b) >> 1;
      if (rec_less(recs[lo + mid], my)) a = mid + 1;
      else b = mid;
    }
    rank += a;
  }
  orig[rank] = (int64_t)my.idx;
  if (D == 2) {
    coords[rank] = (double)my.k2 * 0x1.0p-53;
    coords[N + rank] = (double)(my.k1 - my.k2) * 0x1.0p-53;
  } else {
    for (int q = 0; q < D; ++q) coords[(int64_t)q * N + rank] = raw[(int64_t)q * N + my.idx];
  }
}

template <int D>
__global__ __launch_bounds__(256) void k_rank_scatter(
    const SortRec* __restrict__ recs, int64_t N, const double* __restrict__ raw,
    double* __restrict__ coords, int64_t* __restrict__ orig) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < N) rank_scatter_one<D>(recs, N, raw, coords, orig, e);
}

__global__ __launch_bounds__(256) void k_fill_recs(SortRec* __restrict__ recs,
                                                   int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < n) {
    recs[e].k1 = ~0ull;
    recs[e].k2 = ~0ull;
    recs[e].idx = ~0ull;
  }
}

// ---- batched ensembles ------------------------------------------------------
// One workgroup draws one whole set.  In 4D it walks the candidates
// kBatchSprinkleThreads at a time, ranks the accepted ones with wave ballots
// and stops, all lanes together, as soon as N are accepted: the same first N
// accepted candidates, in candidate order, as the single-set path.  A 4D set
// of 4096 elements needs about 31 000 candidates (the diamond fills pi/24 of
// its bounding box), so the widest workgroup keeps the longest sets short.
constexpr int kBatchSprinkleThreads = 1024;
__global__ __launch_bounds__(kBatchSprinkleThreads) void k_batch_sprinkle(BatchDev b) {
  constexpr int T = kBatchSprinkleThreads, NW = T / 64;
  __shared__ uint32_t wcnt[NW];
  const BatchSet bs = b.sets[blockIdx.x];
  const int64_t N = bs.N;
  if (N <= 0) return;
  SortRec* recs = b.recs + bs.rec_off;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (bs.d == 2) {
    for (int64_t c = tid; c < N; c += T) {
      uint64_t r[4] = {(uint64_t)c, 0, 0, 0};
      philox10(r, bs.seed, 1);
      const uint64_t a = r[0] >> 11, bb = r[1] >> 11;
      SortRec s;
      s.k1 = a + bb;
      s.k2 = a;
      s.idx = (uint64_t)c;
      recs[c] = s;
    }
    return;
  }
  double* raw = b.raw + bs.raw_off;
  int64_t accepted = 0;
  for (int64_t base = 0; accepted < N; base += T) {
    const int64_t c = base + tid;
    double xyz[4];
    uint64_t kt = 0;
    const bool acc = candidate4d((uint64_t)c, bs.seed, xyz, &kt);
    const uint64_t bal = __ballot(acc);
    const uint32_t below = __builtin_amdgcn_mbcnt_hi(
        (uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
    if (lane == 0) wcnt[wave] = (uint32_t)__popcll(bal);
    __syncthreads();
    uint32_t woff = 0, tot = 0;
#pragma unroll
    for (int q = 0; q < NW; ++q) {
      woff += q < wave ? wcnt[q] : 0u;
      tot += wcnt[q];
    }
    // the same for every lane: keep the loop exit a scalar branch
    tot = __builtin_amdgcn_readfirstlane(tot);
    const int64_t e = accepted + woff + below;
    if (acc && e < N) {
      SortRec s;
      s.k1 = kt;
      s.k2 = 0;
      s.idx = (uint64_t)e;
      recs[e] = s;
      raw[e] = xyz[0];
      raw[N + e] = xyz[1];
      raw[2 * N + e] = xyz[2];
      raw[3 * N + e] = xyz[3];
    }
    accepted += tot;
    __syncthreads();  // wcnt is rewritten next round
  }
}

__global__ __launch_bounds__(1024) void k_batch_tile_sort(BatchDev b) {
  __shared__ SortRec s[kSortTile];
  int64_t set, tile, unused;
  unpack_item(b.sort_items[blockIdx.x], &set, &tile, &unused);
  const BatchSet bs = b.sets[set];
  const int64_t base = tile * kSortTile;
  const int64_t n = bs.N - base < kSortTile ? bs.N - base : kSortTile;
  tile_sort_body(b.recs + bs.rec_off + base, n, s);
}

__global__ __launch_bounds__(256) void k_batch_rank_scatter(BatchDev b) {
  int64_t set, chunk, unused;
  unpack_item(b.elem_items[blockIdx.x], &set, &chunk, &unused);
  const BatchSet bs = b.sets[set];
  const int64_t e = chunk * 256 + threadIdx.x;
  if (e >= bs.N) return;
  if (bs.d == 2)
    rank_scatter_one<2>(b.recs + bs.rec_off, bs.N, nullptr, b.coords + bs.coords_off,
                        b.orig + bs.orig_off, e);
  else
    rank_scatter_one<4>(b.recs + bs.rec_off, bs.N, b.raw + bs.raw_off,
                        b.coords + bs.coords_off, b.orig + bs.orig_off, e);
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

int64_t candidates_4d(int64_t N) {
  const double p = 3.14159265358979323846 / 24.0;
  const double mean = (double)N / p;
  const double sd = __builtin_sqrt(mean * (1.0 - p));
  return (int64_t)(mean + 8.0 * sd) + 256;
}

size_t sprinkle_scratch_bytes(int d, int64_t N, int64_t ncand) {
  size_t b = align256((size_t)N * sizeof(SortRec));
  if (d == 4) {
    const int64_t nblk = (ncand + 255) / 256;
    b += align256((size_t)N * 4 * sizeof(double));
    b += align256((size_t)nblk * sizeof(uint32_t));
    b += align256((size_t)nblk * sizeof(uint64_t));
  }
  return b;
}

hipError_t launch_sprinkle(int d, int64_t N, uint64_t seed, int64_t ncand,
                           double* coords, int64_t* orig, void* scratch,
                           uint64_t* accepted_dev, hipStream_t st) {
  if (N <= 0) return hipSuccess;
  char* p = (char*)scratch;
  SortRec* recs = (SortRec*)p;
  p += align256((size_t)N * sizeof(SortRec));
  const unsigned gN = (unsigned)((N + 255) / 256);
  const double* raw = nullptr;
  if (d == 2) {
    hipLaunchKernelGGL(k_keys2d, dim3(gN), dim3(256), 0, st, N, seed, recs);
  } else {
    double* rawm = (double*)p;
    p += align256((size_t)N * 4 * sizeof(double));
    const int64_t nblk = (ncand + 255) / 256;
    uint32_t* blkcnt = (uint32_t*)p;
    p += align256((size_t)nblk * sizeof(uint32_t));
    uint64_t* offs = (uint64_t*)p;
    hipLaunchKernelGGL(k_fill_recs, dim3(gN), dim3(256), 0, st, recs, N);
    hipLaunchKernelGGL(k_count4d, dim3((unsigned)nblk), dim3(256), 0, st, ncand,
                       seed, blkcnt);
    hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, st, blkcnt, nblk,
                       offs, accepted_dev);
    hipLaunchKernelGGL(k_compact4d, dim3((unsigned)nblk), dim3(256), 0, st,
                       ncand, seed, offs, N, recs, rawm);
    raw = rawm;
  }
  const unsigned ntiles = (unsigned)((N + kSortTile - 1) / kSortTile);
  hipLaunchKernelGGL(k_tile_sort, dim3(ntiles), dim3(1024), 0, st, recs, N);
  if (d == 2)
    hipLaunchKernelGGL(k_rank_scatter<2>, dim3(gN), dim3(256), 0, st, recs, N,
                       raw, coords, orig);
  else
    hipLaunchKernelGGL(k_rank_scatter<4>, dim3(gN), dim3(256), 0, st, recs, N,
                       raw, coords, orig);
  return hipGetLastError();
}

size_t sprinkle_desitter_scratch_bytes(int64_t N) {
  return align256((size_t)N * sizeof(SortRec)) + align256((size_t)N * 3 * sizeof(double));
}

hipError_t launch_sprinkle_desitter(int64_t N, uint64_t seed, double w0, double* coords,
                                    int64_t* orig, void* scratch, hipStream_t st) {
  if (N <= 0) return hipSuccess;
  char* p = (char*)scratch;
  SortRec* recs = (SortRec*)p;
  p += align256((size_t)N * sizeof(SortRec));
  double* raw = (double*)p;
  const unsigned gN = (unsigned)((N + 255) / 256);
  hipLaunchKernelGGL(k_keys_desitter, dim3(gN), dim3(256), 0, st, N, seed, w0, recs, raw);
  const unsigned ntiles = (unsigned)((N + kSortTile - 1) / kSortTile);
  hipLaunchKernelGGL(k_tile_sort, dim3(ntiles), dim3(1024), 0, st, recs, N);
  hipLaunchKernelGGL(k_rank_scatter<3>, dim3(gN), dim3(256), 0, st, recs, N, raw, coords, orig);
  return hipGetLastError();
}

hipError_t launch_batch_sprinkle(const BatchDev& b, hipStream_t st) {
  if (b.nsets <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_sprinkle, dim3((unsigned)b.nsets), dim3(kBatchSprinkleThreads), 0, st, b);
  if (b.n_sort > 0)
    hipLaunchKernelGGL(k_batch_tile_sort, dim3((unsigned)b.n_sort), dim3(1024), 0, st, b);
  if (b.n_elem > 0)
    hipLaunchKernelGGL(k_batch_rank_scatter, dim3((unsigned)b.n_elem), dim3(256), 0, st, b);
  return hipGetLastError();
}

}  // namespace cs
