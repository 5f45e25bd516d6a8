// cs_batch.cpp -- batched ensembles (cs_batch_run) and the count-path tuner.
//
// A batch is planned once per shape (the list of (d, N)): one device arena
// holds every set's coordinates, sort records, matrix and row-block stats,
// plus the work-item tables; the whole launch sequence (sprinkle all sets ->
// sort -> link -> persistent counting kernels over static item lists ->
// per-set action) is captured once in a hipGraph and replayed for every call
// with that shape.  The first call of a shape also tunes it: which count
// kernel each (d, N-bucket) group uses and each kernel's persistent grid.
// Only the per-set seeds change between calls: they are copied into the set
// table before the replay.
#include <hip/hip_runtime.h>

#include <cstdlib>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "cs_internal.h"
#include "cs_runtime.h"

namespace cs {

// ------------------------------------------------------------------ tuner
// Picks the counting path per (d, ceil(log2 N)) by timing the three count
// kernels once on a sprinkled set of that size (up to 32768 elements; larger
// sets reuse the 32768 choice between the two matrix-core paths, since timing
// there costs seconds).  Batches have their own tuner (below).
struct Tuner {
  std::mutex mu;
  std::map<std::pair<int, int>, int> best;        // single sets: (d, bucket) -> path
  std::map<std::pair<int, int>, int> batch_kind;  // batches: (d, bucket) -> count kind
};

static int log2_bucket(int64_t N) {
  int b = 0;
  while (((int64_t)1 << b) < N) ++b;
  return b;
}

static double time_count(cs_ctx* ctx, const uint64_t* bits, int64_t N, int64_t W, int path,
                         uint64_t* ws) {
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  const int64_t nrb = num_row_blocks(N);
  auto once = [&] {
    (void)launch_fill_u64(ws, 0, (size_t)nrb * 6, ctx->stream);
    (void)run_count(bits, N, W, 3, path, ws, ctx->stream);
  };
  once();
  (void)hipEventRecord(e0, ctx->stream);
  for (int r = 0; r < 3; ++r) once();
  (void)hipEventRecord(e1, ctx->stream);
  (void)hipEventSynchronize(e1);
  float ms = 0;
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms;
}

int tuned_path(cs_ctx* ctx, int d, int64_t N) {
  if (N < 64) return CS_PATH_POP;
  if (!ctx->tuner) return choose_path(N, 3);
  // beyond 32768 elements the choice measured at 32768 between the two
  // matrix-core contractions carries over (both scale as N^3 there)
  const bool large = N > 32768;
  const int bucket = large ? 15 : log2_bucket(N);
  {
    std::lock_guard<std::mutex> g(ctx->tuner->mu);
    auto it = ctx->tuner->best.find({d, bucket});
    if (it != ctx->tuner->best.end())
      return large && it->second == CS_PATH_POP ? CS_PATH_MFMA : it->second;
  }
  const int64_t Nt = (int64_t)1 << bucket;
  int path = choose_path(Nt, 3);
  cs_set* s = nullptr;
  if (cs_sprinkle(ctx, d, Nt, 0x7475ull, &s) == CS_OK && cs_link(ctx, s) == CS_OK) {
    DevBuf ws(ctx->pool, (size_t)num_row_blocks(Nt) * 6 * 8);
    if (ws.p) {
      double best = 1e300;
      for (int p : {CS_PATH_POP, CS_PATH_MFMA, CS_PATH_MFMA_FP4}) {
        const double t = time_count(ctx, s->bits, Nt, s->W, p, (uint64_t*)ws.p);
        if (t < best) {
          best = t;
          path = p;
        }
      }
    }
  }
  if (s) cs_set_free(s);
  (void)hipGetLastError();
  std::lock_guard<std::mutex> g(ctx->tuner->mu);
  ctx->tuner->best[{d, bucket}] = path;
  return large && path == CS_PATH_POP ? CS_PATH_MFMA : path;
}

void destroy_tuner(Tuner* t) { delete t; }
Tuner* new_tuner() { return new Tuner(); }

// ------------------------------------------------------------------ plans
// Count kernels of a batch, one persistent launch each.
enum { kKindPop = 1, kKindBig = 2, kKindSmall = 3 };

struct BatchPlan {
  std::vector<std::pair<int, int64_t>> shape;  // (d, N); d = 0 marks an invalid request
  std::vector<BatchSet> sets;                  // .path holds the set's count kind
  void* arena = nullptr;
  size_t arena_bytes = 0;
  BatchDev dev{};
  BatchSet* sets_dev = nullptr;
  BatchSet* sets_pinned = nullptr;
  cs_result* results_pinned = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint64_t* item_buf[4] = {nullptr, nullptr, nullptr, nullptr};  // per kind, capacity below
  size_t item_cap[4] = {0, 0, 0, 0};
  int grid[4] = {0, 0, 0, 0};
  int64_t stats_words = 0;
  bool tuned = false;
  cs_batch_info info{};
};

struct BatchState {
  std::list<std::unique_ptr<BatchPlan>> plans;  // most recent first
  BatchPlan* last = nullptr;
};

static void free_plan(cs_ctx* ctx, BatchPlan* p) {
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->exec = nullptr;
  p->graph = nullptr;
  if (p->sets_pinned) (void)hipHostFree(p->sets_pinned);
  if (p->results_pinned) (void)hipHostFree(p->results_pinned);
  ctx->pool.release(p->arena);
}

void destroy_batch_state(cs_ctx* ctx) {
  if (!ctx->batch) return;
  (void)hipStreamSynchronize(ctx->stream);
  for (auto& p : ctx->batch->plans) free_plan(ctx, p.get());
  ctx->batch->plans.clear();
  ctx->batch.reset();
}

static void delete_batch_state(BatchState* b) { delete b; }

static size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

// Work items of one set for a count kind, with a cost for the longest-first
// order: the 4-word chunks (256 columns) a matrix-core tile contracts,
// scaled by its pairs, or the words a popcount tile reads.
static void set_items(int s, int64_t N, int kind, std::vector<std::pair<int64_t, uint64_t>>& out) {
  if (N < 2) return;
  if (kind == kKindBig) {
    const int64_t nb = (N + 255) / 256;
    for (int64_t a = 0; a < nb; ++a)
      for (int64_t b = a; b < nb; ++b) out.push_back({16 * (b - a + 1) + 4, pack_item(s, a, b)});
  } else if (kind == kKindSmall) {
    const int64_t nb = (N + 127) / 128;
    for (int64_t a = 0; a < nb; ++a)
      for (int64_t b = a; b < nb; ++b) out.push_back({4 * (b / 2 - a / 2 + 1) + 2, pack_item(s, a, b)});
  } else {
    const int64_t nb = (N + 63) / 64;
    for (int64_t a = 0; a < nb; ++a)
      for (int64_t b = a; b < nb; ++b) out.push_back({b - a + 1 + 2, pack_item(s, a, b)});
  }
}

static std::vector<uint64_t> sorted_items(std::vector<std::pair<int64_t, uint64_t>>& v) {
  std::stable_sort(v.begin(), v.end(),
                   [](const std::pair<int64_t, uint64_t>& x, const std::pair<int64_t, uint64_t>& y) {
                     return x.first > y.first;
                   });
  std::vector<uint64_t> r;
  r.reserve(v.size());
  for (auto& x : v) r.push_back(x.second);
  return r;
}

static int bucket_of(int64_t N) {
  int b = 0;
  while (((int64_t)1 << b) < N) ++b;
  return b;
}

// A set's count kind: the tuner's choice for its (d, bucket) on this
// context, else a first guess.
static int kind_of(cs_ctx* ctx, int d, int64_t N) {
  if (N < 64) return kKindPop;
  {
    std::lock_guard<std::mutex> g(ctx->tuner->mu);
    auto it = ctx->tuner->batch_kind.find({d, bucket_of(N)});
    if (it != ctx->tuner->batch_kind.end()) return it->second;
  }
  return N <= 1024 ? kKindSmall : kKindBig;
}

static int default_grid(cs_ctx* ctx, int kind, int64_t items) {
  const int64_t g = (int64_t)ctx->num_cu * batch_count_max_blocks(kind);
  return (int)std::max<int64_t>(1, std::min<int64_t>(items, g));
}

// Upload the count items of every set's kind into the plan's item buffers.
static hipError_t upload_items(cs_ctx* ctx, BatchPlan* p) {
  std::vector<std::pair<int64_t, uint64_t>> v[4];
  for (size_t s = 0; s < p->sets.size(); ++s)
    set_items((int)s, p->sets[s].N, p->sets[s].path, v[p->sets[s].path]);
  hipError_t e = hipSuccess;
  int64_t n[4] = {0, 0, 0, 0};
  for (int k = 1; k <= 3; ++k) {
    const std::vector<uint64_t> items = sorted_items(v[k]);
    n[k] = (int64_t)items.size();
    if (e == hipSuccess && !items.empty())
      e = hipMemcpyAsync(p->item_buf[k], items.data(), items.size() * 8, hipMemcpyHostToDevice,
                         ctx->stream);
    // the copy reads host memory that ends with this scope
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  }
  p->dev.n_pop = n[kKindPop];
  p->dev.n_mfma = n[kKindBig];
  p->dev.n_mfma128 = n[kKindSmall];
  for (int k = 1; k <= 3; ++k) p->grid[k] = default_grid(ctx, k, n[k]);
  return e;
}

static hipError_t launch_counts(const BatchDev& dv, const int* grid, hipStream_t st) {
  hipError_t e = launch_batch_count_mfma(dv, grid[kKindBig], st);
  if (e == hipSuccess) e = launch_batch_count_mfma128(dv, grid[kKindSmall], st);
  if (e == hipSuccess) e = launch_batch_count_pop(dv, grid[kKindPop], st);
  return e;
}

static cs_status capture(cs_ctx* ctx, BatchPlan* p) {
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->exec = nullptr;
  p->graph = nullptr;
  hipStream_t st = ctx->stream;
  const BatchDev& dv = p->dev;
  hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "cs_batch_run: begin capture");
  hipError_t le = launch_fill_u64(dv.stats, 0, (size_t)p->stats_words, st);
  if (le == hipSuccess) le = launch_batch_sprinkle(dv, st);
  if (le == hipSuccess) le = launch_batch_link(dv, st);
  if (le == hipSuccess) le = launch_counts(dv, p->grid, st);
  if (le == hipSuccess) le = launch_batch_finish(dv, st);
  e = hipStreamEndCapture(st, &p->graph);
  if (le != hipSuccess) return hip_fail(le, "cs_batch_run: capture launch");
  if (e != hipSuccess) return hip_fail(e, "cs_batch_run: end capture");
  e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) return hip_fail(e, "cs_batch_run: instantiate");
  return CS_OK;
}

// Lay out the arena, build the item tables and capture the graph.
static cs_status build_plan(cs_ctx* ctx, BatchPlan* p) {
  const int nsets = (int)p->shape.size();
  p->sets.resize((size_t)nsets);
  int64_t c_off = 0, o_off = 0, r_off = 0, raw_off = 0, b_off = 0, s_off = 0;
  size_t cap[4] = {0, 0, 0, 0};
  std::vector<uint64_t> sort_items, elem_items, link_items;
  for (int s = 0; s < nsets; ++s) {
    BatchSet& bs = p->sets[(size_t)s];
    const int d = p->shape[(size_t)s].first;
    const int64_t N = d ? p->shape[(size_t)s].second : 0;
    bs.d = d ? d : 2;
    bs.N = N;
    bs.W = row_words(N);
    bs.seed = 0;
    bs.path = kind_of(ctx, bs.d, N);
    bs.coords_off = c_off;
    bs.orig_off = o_off;
    bs.rec_off = r_off;
    bs.raw_off = raw_off;
    bs.bits_off = b_off;
    bs.stats_off = s_off;
    c_off += bs.d * N;
    o_off += N;
    r_off += N;
    raw_off += bs.d == 4 ? 4 * N : 0;
    b_off += N * bs.W;
    s_off += std::max<int64_t>(num_row_blocks(N), 1) * 6;
    if (N <= 0) continue;
    for (int64_t t = 0; t < (N + kSortTile - 1) / kSortTile; ++t) sort_items.push_back(pack_item(s, t, 0));
    for (int64_t c = 0; c < (N + 255) / 256; ++c) elem_items.push_back(pack_item(s, c, 0));
    int64_t nrt = 0, nct = 0;
    (void)batch_link_tiles(N, bs.W, &nrt, &nct);
    for (int64_t ti = 0; ti < nrt; ++ti)
      for (int64_t tk = batch_link_first_col(ti); tk < nct; ++tk) link_items.push_back(pack_item(s, ti, tk));
    // item capacity: enough for any kind the tuner may pick
    for (int k = 1; k <= 3; ++k) {
      std::vector<std::pair<int64_t, uint64_t>> v;
      set_items(s, N, N < 64 ? kKindPop : k, v);
      cap[k] += v.size();
    }
  }
  p->stats_words = s_off;

  // arena layout
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += a256(bytes ? bytes : 8);
    return o;
  };
  const size_t o_sets = take((size_t)nsets * sizeof(BatchSet));
  const size_t o_coords = take((size_t)c_off * 8);
  const size_t o_orig = take((size_t)o_off * 8);
  const size_t o_recs = take((size_t)r_off * sizeof(SortRec));
  const size_t o_raw = take((size_t)raw_off * 8);
  const size_t o_bits = take((size_t)b_off * 8);
  const size_t o_stats = take((size_t)s_off * 8);
  const size_t o_sort = take(sort_items.size() * 8);
  const size_t o_elem = take(elem_items.size() * 8);
  const size_t o_link = take(link_items.size() * 8);
  size_t o_items[4] = {0, 0, 0, 0};
  for (int k = 1; k <= 3; ++k) o_items[k] = take(cap[k] * 8);
  const size_t o_res = take((size_t)nsets * sizeof(cs_result));
  p->arena_bytes = off;
  p->arena = ctx->pool.alloc(off);
  if (!p->arena) return fail(CS_ENOMEM, "cs_batch_run: batch of %llu bytes exceeds the HBM budget",
                             (unsigned long long)off);
  char* A = (char*)p->arena;
  BatchDev& dv = p->dev;
  dv.nsets = nsets;
  p->sets_dev = (BatchSet*)(A + o_sets);
  dv.sets = p->sets_dev;
  dv.coords = (double*)(A + o_coords);
  dv.orig = (int64_t*)(A + o_orig);
  dv.recs = (SortRec*)(A + o_recs);
  dv.raw = (double*)(A + o_raw);
  dv.bits = (uint64_t*)(A + o_bits);
  dv.stats = (uint64_t*)(A + o_stats);
  dv.sort_items = (const uint64_t*)(A + o_sort);
  dv.n_sort = (int64_t)sort_items.size();
  dv.elem_items = (const uint64_t*)(A + o_elem);
  dv.n_elem = (int64_t)elem_items.size();
  dv.link_items = (const uint64_t*)(A + o_link);
  dv.n_link = (int64_t)link_items.size();
  for (int k = 1; k <= 3; ++k) {
    p->item_buf[k] = (uint64_t*)(A + o_items[k]);
    p->item_cap[k] = cap[k];
  }
  dv.pop_items = p->item_buf[kKindPop];
  dv.mfma_items = p->item_buf[kKindBig];
  dv.mfma128_items = p->item_buf[kKindSmall];
  dv.results = (cs_result*)(A + o_res);
  dv.c4 = 4.0 / std::sqrt(6.0);

  hipStream_t st = ctx->stream;
  hipError_t e = hipSuccess;
  auto up = [&](size_t o, const void* src, size_t bytes) {
    if (e == hipSuccess && bytes) e = hipMemcpyAsync(A + o, src, bytes, hipMemcpyHostToDevice, st);
  };
  up(o_sort, sort_items.data(), sort_items.size() * 8);
  up(o_elem, elem_items.data(), elem_items.size() * 8);
  up(o_link, link_items.data(), link_items.size() * 8);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e == hipSuccess) e = upload_items(ctx, p);
  if (e != hipSuccess) return hip_fail(e, "cs_batch_run: upload");

  if (hipHostMalloc((void**)&p->sets_pinned, (size_t)std::max(nsets, 1) * sizeof(BatchSet)) != hipSuccess ||
      hipHostMalloc((void**)&p->results_pinned, (size_t)std::max(nsets, 1) * sizeof(cs_result)) != hipSuccess)
    return fail(CS_ENOMEM, "cs_batch_run: pinned staging");
  return capture(ctx, p);
}

// ------------------------------------------------------------------ tuning
// Time the count kernels alone on the batch's matrices (already linked by a
// replay): the stats are cleared by a fill kernel, the launches bracketed by
// events; best of `reps`.
static double time_counts(cs_ctx* ctx, BatchPlan* p, const BatchDev& dv, const int* grid, int reps) {
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  double best = 1e300;
  for (int r = 0; r < reps; ++r) {
    (void)launch_fill_u64(dv.stats, 0, (size_t)p->stats_words, ctx->stream);
    (void)hipEventRecord(e0, ctx->stream);
    (void)launch_counts(dv, grid, ctx->stream);
    (void)hipEventRecord(e1, ctx->stream);
    (void)hipEventSynchronize(e1);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    best = std::min(best, (double)ms);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return best;
}

static hipError_t read_stats(cs_ctx* ctx, BatchPlan* p, std::vector<uint64_t>& out) {
  out.resize((size_t)p->stats_words);
  hipError_t e = hipMemcpyAsync(out.data(), p->dev.stats, out.size() * 8, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  return e;
}

// The batch autotuner.  For every (d, ceil(log2 N)) group of sets not seen
// before on this context, the popcount kernel (64-row tiles) and the
// matrix-core kernel with 128- and 256-row tiles each count that group's
// sets of this batch on their own; the fastest kind is kept for the group
// (cached per context).  Every candidate must reproduce the first guess's
// counts exactly, else the batch fails.  Then each count kernel's persistent
// grid is chosen among 1, 2 and the resident maximum of workgroups per CU.
static cs_status tune(cs_ctx* ctx, BatchPlan* p) {
  std::vector<uint64_t> ref, got;
  hipError_t e = read_stats(ctx, p, ref);
  if (e != hipSuccess) return hip_fail(e, "cs_batch_run: tuner read");
  const int nsets = (int)p->sets.size();
  p->info.count_ms_untuned = time_counts(ctx, p, p->dev, p->grid, 3);

  std::map<std::pair<int, int>, std::vector<int>> groups;
  for (int s = 0; s < nsets; ++s)
    if (p->sets[(size_t)s].N >= 64 && p->shape[(size_t)s].first != 0)
      groups[{p->sets[(size_t)s].d, bucket_of(p->sets[(size_t)s].N)}].push_back(s);
  for (auto& g : groups) {
    {
      std::lock_guard<std::mutex> lk(ctx->tuner->mu);
      if (ctx->tuner->batch_kind.count(g.first)) continue;
    }
    int best_kind = kKindBig;
    double best = 1e300;
    for (int kind : {kKindPop, kKindSmall, kKindBig}) {
      std::vector<std::pair<int64_t, uint64_t>> v;
      for (int s : g.second) set_items(s, p->sets[(size_t)s].N, kind, v);
      const std::vector<uint64_t> items = sorted_items(v);
      if (items.empty() || items.size() > p->item_cap[kind]) continue;
      BatchDev dv = p->dev;
      dv.n_pop = kind == kKindPop ? (int64_t)items.size() : 0;
      dv.n_mfma = kind == kKindBig ? (int64_t)items.size() : 0;
      dv.n_mfma128 = kind == kKindSmall ? (int64_t)items.size() : 0;
      e = hipMemcpyAsync(p->item_buf[kind], items.data(), items.size() * 8, hipMemcpyHostToDevice,
                         ctx->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
      if (e != hipSuccess) return hip_fail(e, "cs_batch_run: tuner upload");
      int grid[4] = {1, 1, 1, 1};
      grid[kind] = default_grid(ctx, kind, (int64_t)items.size());
      const double ms = time_counts(ctx, p, dv, grid, 2);
      e = read_stats(ctx, p, got);
      if (e != hipSuccess) return hip_fail(e, "cs_batch_run: tuner read");
      for (int s : g.second) {
        const BatchSet& bs = p->sets[(size_t)s];
        const int64_t nw = std::max<int64_t>(num_row_blocks(bs.N), 1) * 6;
        if (!std::equal(got.begin() + bs.stats_off, got.begin() + bs.stats_off + nw, ref.begin() + bs.stats_off))
          return fail(CS_EDEVICE, "cs_batch_run: count kind %d disagrees with the first guess on set %d", kind, s);
      }
      if (ms < best) {
        best = ms;
        best_kind = kind;
      }
    }
    std::lock_guard<std::mutex> lk(ctx->tuner->mu);
    ctx->tuner->batch_kind[g.first] = best_kind;
  }
  for (int s = 0; s < nsets; ++s) p->sets[(size_t)s].path = kind_of(ctx, p->sets[(size_t)s].d, p->sets[(size_t)s].N);
  e = upload_items(ctx, p);
  if (e != hipSuccess) return hip_fail(e, "cs_batch_run: tuner upload");
  // persistent grid per count kernel
  for (int kind : {kKindPop, kKindSmall, kKindBig}) {
    const int64_t n = kind == kKindPop ? p->dev.n_pop : kind == kKindBig ? p->dev.n_mfma : p->dev.n_mfma128;
    if (n == 0) continue;
    const int occ = batch_count_max_blocks(kind);
    double best = 1e300;
    int best_grid = p->grid[kind];
    for (int per_cu : {1, 2, occ}) {
      if (per_cu > occ) continue;
      BatchDev dv = p->dev;
      if (kind != kKindPop) dv.n_pop = 0;
      if (kind != kKindBig) dv.n_mfma = 0;
      if (kind != kKindSmall) dv.n_mfma128 = 0;
      int grid[4] = {1, 1, 1, 1};
      grid[kind] = (int)std::max<int64_t>(1, std::min<int64_t>(n, (int64_t)per_cu * ctx->num_cu));
      const double ms = time_counts(ctx, p, dv, grid, 2);
      if (ms < best) {
        best = ms;
        best_grid = grid[kind];
      }
    }
    p->grid[kind] = best_grid;
  }
  p->info.count_ms_tuned = time_counts(ctx, p, p->dev, p->grid, 3);
  e = read_stats(ctx, p, got);
  if (e != hipSuccess) return hip_fail(e, "cs_batch_run: tuner read");
  if (got != ref) return fail(CS_EDEVICE, "cs_batch_run: tuned counts disagree with the first guess");
  cs_status rc = capture(ctx, p);
  if (rc != CS_OK) return rc;
  p->tuned = true;
  return CS_OK;
}

static void fill_info(BatchPlan* p) {
  cs_batch_info& in = p->info;
  in.sets_pop = in.sets_mfma256 = in.sets_mfma128 = 0;
  for (size_t s = 0; s < p->sets.size(); ++s) {
    if (p->shape[s].first == 0 || p->sets[s].N < 2) continue;
    const int k = p->sets[s].path;
    if (k == kKindPop)
      ++in.sets_pop;
    else if (k == kKindBig)
      ++in.sets_mfma256;
    else
      ++in.sets_mfma128;
  }
  in.grid_pop = p->dev.n_pop ? p->grid[kKindPop] : 0;
  in.grid_mfma256 = p->dev.n_mfma ? p->grid[kKindBig] : 0;
  in.grid_mfma128 = p->dev.n_mfma128 ? p->grid[kKindSmall] : 0;
}

}  // namespace cs

using namespace cs;

extern "C" cs_status cs_batch_run(cs_ctx* ctx, int nsets, const cs_req* reqs, cs_result* out) {
  if (!ctx || nsets < 0 || (nsets > 0 && (!reqs || !out))) return fail(CS_EINVAL, "cs_batch_run: bad arguments");
  if (nsets == 0) return CS_OK;
  (void)hipSetDevice(ctx->device);
  if (!ctx->batch) {
    ctx->batch = std::unique_ptr<BatchState, void (*)(BatchState*)>(new BatchState(), delete_batch_state);
  }
  std::vector<std::pair<int, int64_t>> shape((size_t)nsets);
  for (int s = 0; s < nsets; ++s) {
    const cs_req& r = reqs[s];
    const bool ok = (r.d == 2 || r.d == 4) && r.N >= 0 && r.N <= CS_BATCH_NMAX;
    shape[(size_t)s] = ok ? std::make_pair((int)r.d, (int64_t)r.N) : std::make_pair(0, (int64_t)0);
  }
  auto& plans = ctx->batch->plans;
  BatchPlan* p = nullptr;
  for (auto it = plans.begin(); it != plans.end(); ++it) {
    if ((*it)->shape == shape) {
      plans.splice(plans.begin(), plans, it);
      p = plans.front().get();
      break;
    }
  }
  if (!p) {
    while (plans.size() >= 4) {
      if (ctx->batch->last == plans.back().get()) ctx->batch->last = nullptr;
      free_plan(ctx, plans.back().get());
      plans.pop_back();
    }
    auto np = std::make_unique<BatchPlan>();
    np->shape = shape;
    cs_status rc = build_plan(ctx, np.get());
    if (rc != CS_OK) {
      free_plan(ctx, np.get());
      return rc;
    }
    plans.push_front(std::move(np));
    p = plans.front().get();
  }
  ctx->batch->last = p;
  for (int s = 0; s < nsets; ++s) {
    p->sets_pinned[s] = p->sets[(size_t)s];
    p->sets_pinned[s].seed = reqs[s].seed;
  }
  hipStream_t st = ctx->stream;
  hipError_t e = hipMemcpyAsync(p->sets_dev, p->sets_pinned, (size_t)nsets * sizeof(BatchSet),
                                hipMemcpyHostToDevice, st);
  if (e == hipSuccess && !p->tuned) {
    // first run of this shape: replay the first guess, then tune on its matrices
    e = hipGraphLaunch(p->exec, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "cs_batch_run: replay");
    cs_status rc = tune(ctx, p);
    if (rc != CS_OK) {
      // the plan's item lists and graph are half rewritten: drop it
      ctx->batch->last = nullptr;
      free_plan(ctx, p);
      plans.pop_front();
      return rc;
    }
  }
  if (e == hipSuccess) e = hipGraphLaunch(p->exec, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(p->results_pinned, p->dev.results, (size_t)nsets * sizeof(cs_result),
                       hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "cs_batch_run: replay");
  fill_info(p);
  for (int s = 0; s < nsets; ++s) {
    out[s] = p->results_pinned[s];
    if (shape[(size_t)s].first == 0) {
      std::memset(&out[s], 0, sizeof(cs_result));
      out[s].status = CS_EINVAL;
    }
  }
  return CS_OK;
}

extern "C" cs_status cs_batch_last_info(cs_ctx* ctx, cs_batch_info* out) {
  if (!ctx || !out) return fail(CS_EINVAL, "cs_batch_last_info: NULL argument");
  if (!ctx->batch || !ctx->batch->last) return fail(CS_EINVAL, "cs_batch_last_info: no batch has run");
  *out = ctx->batch->last->info;
  return CS_OK;
}
