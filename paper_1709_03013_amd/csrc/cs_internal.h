// cs_internal.h -- declarations shared by the library's translation units.
//
// Layout conventions (see include/cs.h): coordinates are SoA float64, the
// matrix is N rows of W uint64 words, symmetric, zero diagonal, zero padding.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "cs.h"

namespace cs {

// One record of the time sort: primary key, secondary key, generation index.
// 2D: k1 = a + b, k2 = a (u = a 2^-53, v = b 2^-53, t = (a+b) 2^-54 exactly).
// 4D: k1 = r0 >> 11 (t = k1 2^-53), k2 = 0.  idx makes every key unique.
struct SortRec {
  uint64_t k1;
  uint64_t k2;
  uint64_t idx;
};

constexpr int kSortTile = 2048;  // records sorted per workgroup in LDS
// Full-histogram counting keeps bins 0..kLdsBins-1 in LDS per workgroup and
// adds larger interval sizes straight to the row-block stats in HBM.
constexpr int kLdsBins = 8192;
constexpr int kRowBlock = CS_ROW_BLOCK;

inline int64_t row_words(int64_t N) {
  int64_t w = (N + 63) / 64;
  return (w + 3) / 4 * 4;
}

// Number of Philox candidates drawn for N accepted 4D points: the mean N/p
// (p = pi/24, the acceptance probability) plus 8 standard deviations plus 256.
int64_t candidates_4d(int64_t N);

// ---- launchers (all asynchronous on `st`) --------------------------------
// Sprinkle + sort: writes sorted SoA coords (d*N) and generation indices.
// `scratch` must hold sprinkle_scratch_bytes(d, N, ncand) bytes.  For 4D the
// number of accepted candidates is written to *accepted_dev (device); the
// caller checks it against N (fewer means draw more candidates).
size_t sprinkle_scratch_bytes(int d, int64_t N, int64_t ncand);
hipError_t launch_sprinkle(int d, int64_t N, uint64_t seed, int64_t ncand,
                           double* coords, int64_t* orig, void* scratch,
                           uint64_t* accepted_dev, hipStream_t st);

// (1+1) de Sitter slab: sorted SoA (w = tan eta, x, y), 3*N doubles.
size_t sprinkle_desitter_scratch_bytes(int64_t N);
hipError_t launch_sprinkle_desitter(int64_t N, uint64_t seed, double w0, double* coords,
                                    int64_t* orig, void* scratch, hipStream_t st);

// Link kinds: 2 and 4 = flat diamonds (d rows of coordinates), kLinkDeSitter
// = the (1+1) de Sitter slab (rows w, x, y).
constexpr int kLinkDeSitter = 3;

// Link: bits must hold N*W words; every word of every row is written.
// work: link_workspace_bytes(d, N) bytes of device scratch (2D: the sorted
// block tables; nothing for the other kinds, work may be null), in use until
// the link has finished on `st`.
size_t link_workspace_bytes(int d, int64_t N);
hipError_t launch_link(int d, int64_t N, const double* coords, uint64_t* bits,
                       int64_t W, void* work, hipStream_t st);

// Link tiles of one set in a batch: *nrt row tiles, *nct column tiles; the
// set's items are (ti, tk) for every ti < *nrt and batch_link_first_col(ti)
// <= tk < *nct.  Returns their number.
int64_t batch_link_tiles(int64_t N, int64_t W, int64_t* nrt, int64_t* nct);
int64_t batch_link_first_col(int64_t ti);

// Fill n uint64 words with v (a kernel, so it can sit in a captured graph).
hipError_t launch_fill_u64(uint64_t* p, uint64_t v, size_t n, hipStream_t st);

// Counting.  rb_stats: nrb*(kmax+3) words, zero on entry; receives per
// row-block histograms, R and sum of interior counts.
int64_t num_row_blocks(int64_t N);
hipError_t launch_count_pop(const uint64_t* bits, int64_t N, int64_t W,
                            int kmax, uint64_t* rb_stats, hipStream_t st);
hipError_t launch_count_mfma(const uint64_t* bits, int64_t N, int64_t W,
                             int kmax, uint64_t* rb_stats, hipStream_t st);
hipError_t launch_count_mfma_fp4(const uint64_t* bits, int64_t N, int64_t W,
                                 int kmax, uint64_t* rb_stats, hipStream_t st);
// Sum the row-block stats into tot (kmax+3 words).
hipError_t launch_reduce_rows(const uint64_t* rb_stats, int64_t nrb,
                              int kmax, uint64_t* tot, hipStream_t st);
// Saturating count of the local abundances (N_0..N_3 and R only).  A tile
// of 64x64 pairs (row blocks bi <= bj) counts the chunk [c0, c1) of C words
// in the middle of the words strictly between its blocks, then the rest of
// the staged window [w0, w1) (E more words on each side, clipped to
// [bi, bj]), then the pairs' remaining words from HBM; tiles with
// bj - bi + 1 <= C + 2 count all their words in the chunk.
constexpr int kSatWin = 16;      // most words a tile stages (C + 2E, or C + 2)
// C and E of the library's count: at 2D N = 2^17 (C, E) = (4, 6) took 35 ms,
// (8, 4) 32 ms, (12, 2) 32 ms, (14, 1) 33 ms; every setting gives the same
// counts (the staged window only decides which words are read first).
constexpr int kSatChunk = 8;
constexpr int kSatMargin = 4;
static_assert(kSatChunk >= 1 && kSatChunk + 2 * kSatMargin <= kSatWin, "bad window");
constexpr int kSatBlkWords = 8;  // per block of 64 labels: N_0..N_3, R, pairs continued from HBM
struct SatWin {
  int64_t c0, c1, w0, w1;
};
__host__ __device__ inline SatWin sat_window(int64_t bi, int64_t bj, int C, int E) {
  SatWin s;
  if (bj - bi + 1 <= C + 2) {
    s.c0 = s.w0 = bi;
    s.c1 = s.w1 = bj + 1;
    return s;
  }
  const int64_t g = bj - bi - 1;  // words strictly between the blocks (> C)
  s.c0 = bi + 1 + (g - C) / 2;
  s.c1 = s.c0 + C;
  s.w0 = s.c0 - E > bi ? s.c0 - E : bi;
  s.w1 = s.c1 + E < bj + 1 ? s.c1 + E : bj + 1;
  return s;
}
// Per-block counters: one 64-byte slot per block of 64 labels.
uint64_t sat_workspace_bytes(int64_t N);
// out receives 6 words: N_0..N_3, R, pairs continued from HBM.
hipError_t launch_count_sat(const uint64_t* bits, int64_t N, int64_t W, int C, int E,
                            uint64_t* blk, uint64_t* out, hipStream_t st);
// Validate an imported matrix: writes 0 to *bad_dev if symmetric, zero
// diagonal, zero padding; nonzero otherwise (bad_dev zeroed by the caller).
hipError_t launch_validate(const uint64_t* bits, int64_t N, int64_t W,
                           uint32_t* bad_dev, hipStream_t st);

// Path choice for CS_PATH_AUTO.
int choose_path(int64_t N, int kmax);

// ---- batched ensembles -----------------------------------------------------
// One set of a batch, as the device sees it.  Offsets index the arena arrays.
struct BatchSet {
  int32_t d;
  int32_t path;        // CS_PATH_POP or CS_PATH_MFMA
  int64_t N, W;
  uint64_t seed;
  int64_t coords_off;  // doubles into coords (d*N)
  int64_t orig_off;    // int64 into orig (N)
  int64_t rec_off;     // records into recs (N)
  int64_t raw_off;     // doubles into raw (4*N, 4D only)
  int64_t bits_off;    // words into bits (N*W)
  int64_t stats_off;   // words into stats (nrb*(kmax+3))
};

// Work items: (set, a, b) packed as set << 40 | a << 20 | b.
__host__ __device__ inline uint64_t pack_item(int64_t set, int64_t a, int64_t b) {
  return ((uint64_t)set << 40) | ((uint64_t)a << 20) | (uint64_t)b;
}
__host__ __device__ inline void unpack_item(uint64_t it, int64_t* set, int64_t* a, int64_t* b) {
  *set = (int64_t)(it >> 40);
  *a = (int64_t)((it >> 20) & 0xFFFFF);
  *b = (int64_t)(it & 0xFFFFF);
}

struct BatchDev {
  int nsets;
  const BatchSet* sets;
  double* coords;
  int64_t* orig;
  SortRec* recs;
  double* raw;
  uint64_t* bits;
  uint64_t* stats;
  // item tables
  const uint64_t* sort_items;  int64_t n_sort;     // (set, tile, 0)
  const uint64_t* elem_items;  int64_t n_elem;     // (set, chunk of 256, 0)
  const uint64_t* link_items;  int64_t n_link;     // (set, row tile, column tile)
  const uint64_t* pop_items;   int64_t n_pop;      // (set, bi, bj), 64-row blocks
  const uint64_t* mfma_items;  int64_t n_mfma;     // (set, BI, BJ), 256-row blocks
  const uint64_t* mfma128_items; int64_t n_mfma128; // (set, BI, BJ), 128-row blocks
  cs_result* results;
  double c4;                                       // 4/sqrt(6), rounded once on the host
};

hipError_t launch_batch_sprinkle(const BatchDev& b, hipStream_t st);
hipError_t launch_batch_link(const BatchDev& b, hipStream_t st);
hipError_t launch_batch_count_pop(const BatchDev& b, int grid, hipStream_t st);
hipError_t launch_batch_count_mfma(const BatchDev& b, int grid, hipStream_t st);
hipError_t launch_batch_count_mfma128(const BatchDev& b, int grid, hipStream_t st);
// Resident workgroups per CU of a batched count kernel (kind: 1 popcount,
// 2 matrix core with 256-row tiles, 3 with 128-row tiles).
int batch_count_max_blocks(int kind);
int batch_count_pop_max_blocks();
// Once per device before the first count: kernel attributes (LDS limits).
hipError_t init_count_mfma();
hipError_t launch_batch_finish(const BatchDev& b, hipStream_t st);

// BD action from abundances (host): exact int64 bracket, one rounding.
double bd_action(int d, int64_t N, const uint64_t* n);

}  // namespace cs
