// cs_runtime.h -- host-side runtime objects: device memory pool, contexts,
// sets, and the hooks the batched and queued paths attach to a context.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <unordered_map>

#include "cs.h"

namespace cs {

// Caching device allocator with an HBM budget on live bytes.  Blocks up to
// 1 MiB round to 256 B, larger ones to 2 MiB; a free block is reused when it
// is at most 25% larger than the request.  Cached blocks are released when
// a new allocation would push live + cached bytes over the budget.
struct Pool {
  uint64_t budget = 0;
  uint64_t live_bytes = 0;
  uint64_t cached_bytes = 0;
  std::multimap<size_t, void*> free_blocks;
  std::unordered_map<void*, size_t> live;
  std::mutex mu;
  void* alloc(size_t bytes);  // nullptr when over budget or out of memory
  void release(void* p);
  void trim();
  static size_t round_up(size_t b);
  ~Pool();
};

// Scoped pool allocation.
struct DevBuf {
  Pool& pool;
  void* p;
  DevBuf(Pool& pl, size_t bytes) : pool(pl), p(pl.alloc(bytes)) {}
  ~DevBuf() { pool.release(p); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
};

struct BatchState;
struct QueueState;
struct Tuner;

}  // namespace cs

struct cs_ctx {
  int device = 0;
  int num_cu = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  cs::Pool pool;
  std::unique_ptr<cs::BatchState, void (*)(cs::BatchState*)> batch{nullptr, nullptr};
  std::unique_ptr<cs::QueueState, void (*)(cs::QueueState*)> queue{nullptr, nullptr};
  std::unique_ptr<cs::Tuner, void (*)(cs::Tuner*)> tuner{nullptr, nullptr};
};

struct cs_set {
  cs_ctx* ctx = nullptr;
  int d = 0;
  int manifold = 0;          // CS_MANIFOLD_*
  int rows = 0;              // coordinate rows: d, or 3 for de Sitter
  int64_t N = 0, W = 0;
  double* coords = nullptr;  // rows*N SoA, sorted
  int64_t* orig = nullptr;   // generation index of each sorted element
  uint64_t* bits = nullptr;  // N*W words
  void* link_work = nullptr; // 2D link tables (link_workspace_bytes), kept until the set is freed
  bool linked = false;
  int counted_kmax = -1;
  int last_path = 0;  // count path used by the last cs_interval_abundances
  uint64_t n[4] = {0, 0, 0, 0};
  uint64_t R = 0, summ = 0;
};

namespace cs {

cs_status fail(cs_status s, const char* fmt, ...);
cs_status hip_fail(hipError_t e, const char* what);
hipError_t run_count(const uint64_t* bits, int64_t N, int64_t W, int kmax, int path,
                     uint64_t* rb_stats, hipStream_t st);
cs_status count_matrix(cs_ctx* ctx, const uint64_t* bits, int64_t N, int64_t W, int kmax,
                       int path, uint64_t* tot_host, uint64_t* rows_host, hipStream_t st);
void destroy_batch_state(cs_ctx* ctx);
void destroy_tuner(Tuner* t);
Tuner* new_tuner();
// Counting path for a set of d, N on this context (timed once per size bucket).
int tuned_path(cs_ctx* ctx, int d, int64_t N);

}  // namespace cs
