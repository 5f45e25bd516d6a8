// cs_batch.cpp -- batched ensembles (cs_batch_run) and the count-path tuner.
//
// A batch is planned once per shape (the list of (d, N)): one device arena
// holds every set's coordinates, sort records, matrix and row-block stats,
// plus the work-item tables; the whole launch sequence (sprinkle all sets ->
// sort -> link -> persistent counting kernels fed by device queues -> per-set
// action) is captured once in a hipGraph and replayed for every call with
// that shape.  Only the per-set seeds change between calls: they are copied
// into the set table before the replay.
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
// there costs seconds).  The batch path runs sets tuned to either MFMA path
// on its int8 persistent kernel.
struct Tuner {
  std::mutex mu;
  std::map<std::pair<int, int>, int> best;
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
struct BatchPlan {
  std::vector<std::pair<int, int64_t>> shape;  // (d, N); d = 0 marks an invalid request
  std::vector<BatchSet> sets;
  void* arena = nullptr;
  size_t arena_bytes = 0;
  BatchDev dev{};
  BatchSet* sets_dev = nullptr;
  BatchSet* sets_pinned = nullptr;
  cs_result* results_pinned = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int pop_grid = 0, mfma_grid = 0;
};

struct BatchState {
  std::list<std::unique_ptr<BatchPlan>> plans;  // most recent first
};

static void free_plan(cs_ctx* ctx, BatchPlan* p) {
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
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

// Count path of one set in a batch.  A batch is throughput-bound, not
// latency-bound, so the tuner's single-set timings do not apply: every set of
// 64 or more elements goes to the matrix cores (fp4), which on MI355X ran
// the 512-set ensemble in 3.8 ms against 7.8 ms with every set on the
// popcount kernel and 8 ms with the tuner's choices.  CS_BATCH_PATH (timing
// only): 1 = every set on the popcount kernel, 3 = the tuner's choice.
static int batch_path(cs_ctx* ctx, int d, int64_t N) {
  const char* e = getenv("CS_BATCH_PATH");
  const int mode = e ? atoi(e) : 2;
  if (mode == 1) return CS_PATH_POP;
  if (mode == 3) return tuned_path(ctx, d, N);
  return N >= 64 ? CS_PATH_MFMA_FP4 : CS_PATH_POP;
}

// Lay out the arena, build the item tables and capture the graph.
static cs_status build_plan(cs_ctx* ctx, BatchPlan* p) {
  const int nsets = (int)p->shape.size();
  p->sets.resize((size_t)nsets);
  int64_t c_off = 0, o_off = 0, r_off = 0, raw_off = 0, b_off = 0, s_off = 0;
  std::vector<std::pair<int64_t, uint64_t>> pop, mfma;  // (cost, item)
  std::vector<uint64_t> sort_items, elem_items, link_items;
  for (int s = 0; s < nsets; ++s) {
    BatchSet& bs = p->sets[(size_t)s];
    const int d = p->shape[(size_t)s].first;
    const int64_t N = d ? p->shape[(size_t)s].second : 0;
    bs.d = d ? d : 2;
    bs.N = N;
    bs.W = row_words(N);
    bs.seed = 0;
    bs.path = N > 0 ? batch_path(ctx, bs.d, N) : CS_PATH_POP;
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
    for (int64_t ti = 0; ti < (N + 63) / 64; ++ti)
      for (int64_t tw = 0; tw < (bs.W + 63) / 64; ++tw) link_items.push_back(pack_item(s, ti, tw));
    if (N < 2) continue;
    if (bs.path == CS_PATH_MFMA || bs.path == CS_PATH_MFMA_FP4) {
      const int64_t nb = (N + 255) / 256;
      for (int64_t a = 0; a < nb; ++a)
        for (int64_t b = a; b < nb; ++b) mfma.push_back({16 * (b - a + 1) + 4, pack_item(s, a, b)});
    } else {
      const int64_t nb = (N + 63) / 64;
      for (int64_t a = 0; a < nb; ++a)
        for (int64_t b = a; b < nb; ++b) pop.push_back({b - a + 1 + 2, pack_item(s, a, b)});
    }
  }
  auto by_cost = [](const std::pair<int64_t, uint64_t>& x, const std::pair<int64_t, uint64_t>& y) {
    return x.first > y.first;
  };
  std::stable_sort(pop.begin(), pop.end(), by_cost);
  std::stable_sort(mfma.begin(), mfma.end(), by_cost);

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
  const size_t o_pop = take(pop.size() * 8);
  const size_t o_mfma = take(mfma.size() * 8);
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
  dv.pop_items = (const uint64_t*)(A + o_pop);
  dv.n_pop = (int64_t)pop.size();
  dv.mfma_items = (const uint64_t*)(A + o_mfma);
  dv.n_mfma = (int64_t)mfma.size();
  dv.results = (cs_result*)(A + o_res);
  dv.c4 = 4.0 / std::sqrt(6.0);

  std::vector<uint64_t> popv, mfmav;
  for (auto& x : pop) popv.push_back(x.second);
  for (auto& x : mfma) mfmav.push_back(x.second);
  hipStream_t st = ctx->stream;
  hipError_t e = hipSuccess;
  auto up = [&](size_t o, const void* src, size_t bytes) {
    if (e == hipSuccess && bytes) e = hipMemcpyAsync(A + o, src, bytes, hipMemcpyHostToDevice, st);
  };
  up(o_sort, sort_items.data(), sort_items.size() * 8);
  up(o_elem, elem_items.data(), elem_items.size() * 8);
  up(o_link, link_items.data(), link_items.size() * 8);
  up(o_pop, popv.data(), popv.size() * 8);
  up(o_mfma, mfmav.data(), mfmav.size() * 8);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "cs_batch_run: upload");

  if (hipHostMalloc((void**)&p->sets_pinned, (size_t)std::max(nsets, 1) * sizeof(BatchSet)) != hipSuccess ||
      hipHostMalloc((void**)&p->results_pinned, (size_t)std::max(nsets, 1) * sizeof(cs_result)) != hipSuccess)
    return fail(CS_ENOMEM, "cs_batch_run: pinned staging");

  p->pop_grid = (int)std::min<int64_t>(std::max<int64_t>(dv.n_pop, 1), (int64_t)ctx->num_cu * 12);
  p->mfma_grid = (int)std::min<int64_t>(std::max<int64_t>(dv.n_mfma, 1), (int64_t)ctx->num_cu);

  // capture the launch sequence
  e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "cs_batch_run: begin capture");
  hipError_t le = launch_fill_u64(dv.stats, 0, (size_t)s_off, st);
  if (le == hipSuccess) le = launch_batch_sprinkle(dv, st);
  if (le == hipSuccess) le = launch_batch_link(dv, st);
  if (le == hipSuccess) le = launch_batch_count_mfma(dv, p->mfma_grid, st);
  if (le == hipSuccess) le = launch_batch_count_pop(dv, p->pop_grid, st);
  if (le == hipSuccess) le = launch_batch_finish(dv, st);
  e = hipStreamEndCapture(st, &p->graph);
  if (le != hipSuccess) return hip_fail(le, "cs_batch_run: capture launch");
  if (e != hipSuccess) return hip_fail(e, "cs_batch_run: end capture");
  e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) return hip_fail(e, "cs_batch_run: instantiate");
  return CS_OK;
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
  for (int s = 0; s < nsets; ++s) {
    p->sets_pinned[s] = p->sets[(size_t)s];
    p->sets_pinned[s].seed = reqs[s].seed;
  }
  hipStream_t st = ctx->stream;
  hipError_t e = hipMemcpyAsync(p->sets_dev, p->sets_pinned, (size_t)nsets * sizeof(BatchSet),
                                hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipGraphLaunch(p->exec, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(p->results_pinned, p->dev.results, (size_t)nsets * sizeof(cs_result),
                       hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "cs_batch_run: replay");
  for (int s = 0; s < nsets; ++s) {
    out[s] = p->results_pinned[s];
    if (shape[(size_t)s].first == 0) {
      std::memset(&out[s], 0, sizeof(cs_result));
      out[s].status = CS_EINVAL;
    }
  }
  return CS_OK;
}
