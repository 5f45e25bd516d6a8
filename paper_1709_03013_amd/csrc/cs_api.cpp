// cs_api.cpp -- the C ABI of include/cs.h: contexts, sets, the per-set
// path (sprinkle -> link -> count -> action) and the device-pointer tier.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "cs_internal.h"
#include "cs_runtime.h"

using namespace cs;

namespace cs {

thread_local std::string g_last_error;

cs_status fail(cs_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

cs_status hip_fail(hipError_t e, const char* what) {
  return fail(CS_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

double bd_action(int d, int64_t N, const uint64_t* n) {
  if (d == 2) {
    const int64_t K = N - 2 * (int64_t)n[0] + 4 * (int64_t)n[1] - 2 * (int64_t)n[2];
    return 2.0 * (double)K;
  }
  const int64_t K = N - (int64_t)n[0] + 9 * (int64_t)n[1] - 16 * (int64_t)n[2] +
                    8 * (int64_t)n[3];
  const double c = 4.0 / std::sqrt(6.0);
  return c * (double)K;
}

double smeared_action(int64_t N, const uint64_t* hist, int64_t nbins, double eps) {
  // f2(k) = q^k - 2 eps k q^(k-1) + eps^2 (k(k-1)/2) q^(k-2), summed over k
  // ascending with q^k carried by repeated multiplication (Eq. 5).
  const double q = 1.0 - eps;
  double pk = 1.0, pk1 = 0.0, pk2 = 0.0;
  double sum = 0.0;
  for (int64_t k = 0; k < nbins; ++k) {
    const double twoek = (2.0 * eps) * (double)k;
    const double c = (double)(k * (k - 1) / 2);
    const double f = (pk - twoek * pk1) + ((eps * eps) * c) * pk2;
    sum = sum + (double)hist[k] * f;
    pk2 = pk1;
    pk1 = pk;
    pk = pk * q;
  }
  return (2.0 * eps) * ((double)N - (2.0 * eps) * sum);
}

int choose_path(int64_t N, int kmax) {
  (void)kmax;
  // Measured on MI355X: the popcount kernel wins up to N ~ 4096 (launch-bound
  // sizes, less tile waste), the MFMA contraction from N ~ 8192 on.
  return N >= 6144 ? CS_PATH_MFMA : CS_PATH_POP;
}

// ---------------------------------------------------------------- Pool
void* Pool::alloc(size_t bytes) {
  if (bytes == 0) bytes = 256;
  const size_t sz = round_up(bytes);
  std::lock_guard<std::mutex> g(mu);
  if (live_bytes + sz > budget) return nullptr;
  auto it = free_blocks.lower_bound(sz);
  if (it != free_blocks.end() && it->first <= sz + sz / 4) {
    void* p = it->second;
    cached_bytes -= it->first;
    live[p] = it->first;
    live_bytes += it->first;
    free_blocks.erase(it);
    return p;
  }
  // release cached blocks until the new one fits next to the live ones
  while (!free_blocks.empty() && live_bytes + cached_bytes + sz > budget) {
    auto big = std::prev(free_blocks.end());
    (void)hipFree(big->second);
    cached_bytes -= big->first;
    free_blocks.erase(big);
  }
  void* p = nullptr;
  if (hipMalloc(&p, sz) != hipSuccess) {
    (void)hipGetLastError();
    // one more try with the whole cache released
    for (auto& kv : free_blocks) (void)hipFree(kv.second);
    free_blocks.clear();
    cached_bytes = 0;
    if (hipMalloc(&p, sz) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
  }
  live[p] = sz;
  live_bytes += sz;
  return p;
}

void Pool::release(void* p) {
  if (!p) return;
  std::lock_guard<std::mutex> g(mu);
  auto it = live.find(p);
  if (it == live.end()) return;
  live_bytes -= it->second;
  cached_bytes += it->second;
  free_blocks.emplace(it->second, p);
  live.erase(it);
}

void Pool::trim() {
  std::lock_guard<std::mutex> g(mu);
  for (auto& kv : free_blocks) (void)hipFree(kv.second);
  free_blocks.clear();
  cached_bytes = 0;
}

size_t Pool::round_up(size_t b) {
  if (b <= (1u << 20)) return (b + 255) & ~(size_t)255;
  const size_t g = (size_t)2 << 20;
  return (b + g - 1) / g * g;
}

Pool::~Pool() {
  for (auto& kv : free_blocks) (void)hipFree(kv.second);
  for (auto& kv : live) (void)hipFree(kv.first);
}

// Count a matrix into tot (kmax+3 words) and optionally the row-block stats,
// on stream st, using pool memory for the workspace.  Synchronous only in
// the final copies.
cs_status count_matrix(cs_ctx* ctx, const uint64_t* bits, int64_t N, int64_t W,
                       int kmax, int path, uint64_t* tot_host,
                       uint64_t* rows_host, hipStream_t st) {
  const int64_t nrb = num_row_blocks(N);
  const size_t nws = (size_t)(nrb > 0 ? nrb : 1) * (kmax + 3);
  DevBuf ws(ctx->pool, nws * sizeof(uint64_t));
  DevBuf tot(ctx->pool, (size_t)(kmax + 3) * sizeof(uint64_t));
  if (!ws.p || !tot.p) return fail(CS_ENOMEM, "count workspace exceeds budget");
  hipError_t e = launch_fill_u64((uint64_t*)ws.p, 0, nws, st);
  if (e == hipSuccess) e = run_count((const uint64_t*)bits, N, W, kmax, path, (uint64_t*)ws.p, st);
  if (e == hipSuccess) e = launch_reduce_rows((uint64_t*)ws.p, nrb > 0 ? nrb : 1, kmax, (uint64_t*)tot.p, st);
  if (e != hipSuccess) return hip_fail(e, "count launch");
  if (tot_host) e = hipMemcpyAsync(tot_host, tot.p, (size_t)(kmax + 3) * 8, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess && rows_host)
    e = hipMemcpyAsync(rows_host, ws.p, (size_t)nrb * (kmax + 3) * 8, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "count copy");
  return CS_OK;
}

hipError_t run_count(const uint64_t* bits, int64_t N, int64_t W, int kmax, int path,
                     uint64_t* rb_stats, hipStream_t st) {
  if (path == CS_PATH_AUTO) path = choose_path(N, kmax);
  if (path == CS_PATH_MFMA) return launch_count_mfma(bits, N, W, kmax, rb_stats, st);
  if (path == CS_PATH_MFMA_FP4) return launch_count_mfma_fp4(bits, N, W, kmax, rb_stats, st);
  return launch_count_pop(bits, N, W, kmax, rb_stats, st);
}

}  // namespace cs

// =================================================================== ABI
extern "C" {

int64_t cs_row_words(int64_t N) { return N < 0 ? 0 : row_words(N); }

const char* cs_last_error(void) { return g_last_error.c_str(); }

cs_status cs_create(cs_ctx** out, int device, uint64_t hbm_budget_bytes, void* hip_stream) {
  if (!out) return fail(CS_EINVAL, "cs_create: out is NULL");
  *out = nullptr;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev == 0) return fail(CS_EDEVICE, "cs_create: no HIP device");
  if (device < 0 || device >= ndev) return fail(CS_EINVAL, "cs_create: device %d of %d", device, ndev);
  e = hipSetDevice(device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(CS_EUNSUPPORTED, "cs_create: device is %s, library is built for gfx950", prop.gcnArchName);
  e = init_count_mfma();
  if (e != hipSuccess) return hip_fail(e, "count kernel attributes");
  cs_ctx* c = new cs_ctx();
  c->device = device;
  c->num_cu = prop.multiProcessorCount;
  if (hbm_budget_bytes == 0) {
    size_t fr = 0, tot = 0;
    (void)hipMemGetInfo(&fr, &tot);
    hbm_budget_bytes = (uint64_t)(0.9 * (double)fr);
  }
  c->pool.budget = hbm_budget_bytes;
  c->tuner = std::unique_ptr<Tuner, void (*)(Tuner*)>(new_tuner(), destroy_tuner);
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
    c->own_stream = false;
  } else {
    e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete c;
      return hip_fail(e, "hipStreamCreate");
    }
    c->own_stream = true;
  }
  *out = c;
  return CS_OK;
}

void cs_destroy(cs_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  cs_queue_stop(ctx);
  destroy_batch_state(ctx);
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

uint64_t cs_bytes_in_use(const cs_ctx* ctx) { return ctx ? ctx->pool.live_bytes : 0; }

static cs_status new_set(cs_ctx* ctx, int d, int64_t N, cs_set** out, int rows = -1,
                         int manifold = CS_MANIFOLD_DIAMOND) {
  cs_set* s = new cs_set();
  s->ctx = ctx;
  s->d = d;
  s->rows = rows < 0 ? d : rows;
  s->manifold = manifold;
  s->N = N;
  s->W = row_words(N);
  if (N > 0 && s->rows > 0) {
    s->coords = (double*)ctx->pool.alloc((size_t)N * s->rows * sizeof(double));
    s->orig = (int64_t*)ctx->pool.alloc((size_t)N * sizeof(int64_t));
    if (!s->coords || !s->orig) {
      cs_set_free(s);
      return fail(CS_ENOMEM, "set of %lld elements exceeds the HBM budget", (long long)N);
    }
  }
  *out = s;
  return CS_OK;
}

cs_status cs_sprinkle(cs_ctx* ctx, int d, int64_t N, uint64_t seed, cs_set** out) {
  if (!ctx || !out) return fail(CS_EINVAL, "cs_sprinkle: NULL argument");
  *out = nullptr;
  if (d != 2 && d != 4) return fail(CS_EINVAL, "cs_sprinkle: d must be 2 or 4, got %d", d);
  if (N < 0 || N > ((int64_t)1 << 31)) return fail(CS_EINVAL, "cs_sprinkle: bad N %lld", (long long)N);
  (void)hipSetDevice(ctx->device);
  cs_set* s = nullptr;
  cs_status rc = new_set(ctx, d, N, &s);
  if (rc != CS_OK) return rc;
  if (N == 0) {
    *out = s;
    return CS_OK;
  }
  int64_t ncand = d == 4 ? candidates_4d(N) : N;
  for (int attempt = 0; attempt < 8; ++attempt) {
    DevBuf scratch(ctx->pool, sprinkle_scratch_bytes(d, N, ncand));
    DevBuf acc(ctx->pool, sizeof(uint64_t));
    if (!scratch.p || !acc.p) {
      cs_set_free(s);
      return fail(CS_ENOMEM, "cs_sprinkle: scratch exceeds budget");
    }
    hipError_t e = launch_sprinkle(d, N, seed, ncand, s->coords, s->orig, scratch.p,
                                   (uint64_t*)acc.p, ctx->stream);
    if (e != hipSuccess) {
      cs_set_free(s);
      return hip_fail(e, "sprinkle launch");
    }
    if (d == 2) {
      // finish before the scratch returns to the pool: another stream (a
      // queue slot) may be handed the same block next
      e = hipStreamSynchronize(ctx->stream);
      if (e != hipSuccess) {
        cs_set_free(s);
        return hip_fail(e, "sprinkle");
      }
      break;
    }
    uint64_t got = 0;
    e = hipMemcpyAsync(&got, acc.p, 8, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
      cs_set_free(s);
      return hip_fail(e, "sprinkle count");
    }
    if ((int64_t)got >= N) break;
    ncand *= 2;  // far tail: draw more candidates (same counters, same result)
    if (attempt == 7) {
      cs_set_free(s);
      return fail(CS_EDEVICE, "cs_sprinkle: acceptance far below expectation");
    }
  }
  *out = s;
  return CS_OK;
}

cs_status cs_sprinkle_desitter(cs_ctx* ctx, int64_t N, uint64_t seed, double eta0, cs_set** out) {
  if (!ctx || !out) return fail(CS_EINVAL, "cs_sprinkle_desitter: NULL argument");
  *out = nullptr;
  if (!(eta0 > 0.0 && eta0 < 0.78539816339744830962))
    return fail(CS_EINVAL, "cs_sprinkle_desitter: eta0 must be in (0, pi/4), got %g", eta0);
  if (N < 0 || N > ((int64_t)1 << 31)) return fail(CS_EINVAL, "cs_sprinkle_desitter: bad N %lld", (long long)N);
  (void)hipSetDevice(ctx->device);
  cs_set* s = nullptr;
  cs_status rc = new_set(ctx, 2, N, &s, 3, CS_MANIFOLD_DESITTER);
  if (rc != CS_OK) return rc;
  if (N > 0) {
    DevBuf scratch(ctx->pool, sprinkle_desitter_scratch_bytes(N));
    if (!scratch.p) {
      cs_set_free(s);
      return fail(CS_ENOMEM, "cs_sprinkle_desitter: scratch exceeds budget");
    }
    hipError_t e = launch_sprinkle_desitter(N, seed, std::tan(eta0), s->coords, s->orig,
                                            scratch.p, ctx->stream);
    // finish before the scratch returns to the pool
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
      cs_set_free(s);
      return hip_fail(e, "de Sitter sprinkle");
    }
  }
  *out = s;
  return CS_OK;
}

cs_status cs_set_manifold(const cs_set* s, int* manifold, int* coord_rows) {
  if (!s) return fail(CS_EINVAL, "cs_set_manifold: NULL set");
  if (manifold) *manifold = s->manifold;
  if (coord_rows) *coord_rows = s->rows;
  return CS_OK;
}

cs_status cs_set_from_coords(cs_ctx* ctx, int d, int64_t N, const double* coords, cs_set** out) {
  if (!ctx || !out || (N > 0 && !coords)) return fail(CS_EINVAL, "cs_set_from_coords: NULL argument");
  *out = nullptr;
  if (d != 2 && d != 4) return fail(CS_EINVAL, "cs_set_from_coords: d must be 2 or 4");
  if (N < 0 || N > ((int64_t)1 << 31)) return fail(CS_EINVAL, "cs_set_from_coords: bad N");
  (void)hipSetDevice(ctx->device);
  cs_set* s = nullptr;
  cs_status rc = new_set(ctx, d, N, &s);
  if (rc != CS_OK) return rc;
  if (N > 0) {
    std::vector<int64_t> idx((size_t)N);
    for (int64_t i = 0; i < N; ++i) idx[(size_t)i] = i;
    hipError_t e = hipMemcpyAsync(s->coords, coords, (size_t)N * d * 8, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(s->orig, idx.data(), (size_t)N * 8, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
      cs_set_free(s);
      return hip_fail(e, "cs_set_from_coords copy");
    }
  }
  *out = s;
  return CS_OK;
}

cs_status cs_set_from_bitset(cs_ctx* ctx, int d, int64_t N, const uint64_t* rows,
                             int64_t stride_words, int on_device, int validate, cs_set** out) {
  if (!ctx || !out || (N > 0 && !rows)) return fail(CS_EINVAL, "cs_set_from_bitset: NULL argument");
  *out = nullptr;
  if (d != 0 && d != 2 && d != 4) return fail(CS_EINVAL, "cs_set_from_bitset: d must be 0, 2 or 4");
  if (N < 0 || N > ((int64_t)1 << 31)) return fail(CS_EINVAL, "cs_set_from_bitset: bad N");
  const int64_t W = row_words(N);
  if (stride_words < W) return fail(CS_EINVAL, "cs_set_from_bitset: stride %lld < %lld words", (long long)stride_words, (long long)W);
  (void)hipSetDevice(ctx->device);
  cs_set* s = new cs_set();
  s->ctx = ctx;
  s->d = d;
  s->N = N;
  s->W = W;
  if (N > 0) {
    s->bits = (uint64_t*)ctx->pool.alloc((size_t)N * W * 8);
    if (!s->bits) {
      cs_set_free(s);
      return fail(CS_ENOMEM, "cs_set_from_bitset: matrix exceeds budget");
    }
    hipError_t e = hipMemcpy2DAsync(s->bits, (size_t)W * 8, rows, (size_t)stride_words * 8, (size_t)W * 8,
                                    (size_t)N, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                                    ctx->stream);
    if (e != hipSuccess) {
      cs_set_free(s);
      return hip_fail(e, "cs_set_from_bitset copy");
    }
    if (validate) {
      DevBuf bad(ctx->pool, 8);
      if (!bad.p) {
        cs_set_free(s);
        return fail(CS_ENOMEM, "validate flag");
      }
      uint32_t hbad = 0;
      e = launch_fill_u64((uint64_t*)bad.p, 0, 1, ctx->stream);
      if (e == hipSuccess) e = launch_validate(s->bits, N, W, (uint32_t*)bad.p, ctx->stream);
      if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad.p, 4, hipMemcpyDeviceToHost, ctx->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
      if (e != hipSuccess) {
        cs_set_free(s);
        return hip_fail(e, "validate");
      }
      if (hbad) {
        cs_set_free(s);
        return fail(CS_EINVAL, "cs_set_from_bitset: matrix not symmetric, diagonal or padding not zero");
      }
    }
  }
  s->linked = true;
  *out = s;
  return CS_OK;
}

void cs_set_free(cs_set* s) {
  if (!s) return;
  if (s->ctx) {
    (void)hipSetDevice(s->ctx->device);
    (void)hipStreamSynchronize(s->ctx->stream);
    s->ctx->pool.release(s->coords);
    s->ctx->pool.release(s->orig);
    s->ctx->pool.release(s->bits);
    s->ctx->pool.release(s->link_work);
  }
  delete s;
}

cs_status cs_set_info(const cs_set* s, int* d, int64_t* N, int64_t* W, int* linked) {
  if (!s) return fail(CS_EINVAL, "cs_set_info: NULL set");
  if (d) *d = s->d;
  if (N) *N = s->N;
  if (W) *W = s->W;
  if (linked) *linked = s->linked ? 1 : 0;
  return CS_OK;
}

cs_status cs_get_coords(cs_ctx* ctx, const cs_set* s, double* coords, int64_t* orig) {
  if (!ctx || !s) return fail(CS_EINVAL, "cs_get_coords: NULL argument");
  if (!s->coords && s->N > 0) return fail(CS_EINVAL, "cs_get_coords: set has no coordinates");
  (void)hipSetDevice(ctx->device);
  hipError_t e = hipSuccess;
  if (s->N > 0 && coords)
    e = hipMemcpyAsync(coords, s->coords, (size_t)s->N * s->rows * 8, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess && s->N > 0 && orig)
    e = hipMemcpyAsync(orig, s->orig, (size_t)s->N * 8, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  return e == hipSuccess ? CS_OK : hip_fail(e, "cs_get_coords");
}

cs_status cs_get_bitset(cs_ctx* ctx, const cs_set* s, uint64_t* rows) {
  if (!ctx || !s || !rows) return fail(CS_EINVAL, "cs_get_bitset: NULL argument");
  if (!s->linked) return fail(CS_EINVAL, "cs_get_bitset: set is not linked");
  (void)hipSetDevice(ctx->device);
  hipError_t e = hipSuccess;
  if (s->N > 0) e = hipMemcpyAsync(rows, s->bits, (size_t)s->N * s->W * 8, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  return e == hipSuccess ? CS_OK : hip_fail(e, "cs_get_bitset");
}

const uint64_t* cs_set_bitset_dev(const cs_set* s) { return s && s->linked ? s->bits : nullptr; }

int cs_set_count_path(const cs_set* s) { return s ? s->last_path : 0; }

cs_status cs_link(cs_ctx* ctx, cs_set* s) {
  if (!ctx || !s) return fail(CS_EINVAL, "cs_link: NULL argument");
  if (s->linked) return CS_OK;
  if (s->N > 0 && !s->coords) return fail(CS_EINVAL, "cs_link: set has no coordinates");
  (void)hipSetDevice(ctx->device);
  if (s->N > 0) {
    s->bits = (uint64_t*)ctx->pool.alloc((size_t)s->N * s->W * 8);
    if (!s->bits)
      return fail(CS_ENOMEM, "cs_link: matrix of %llu bytes exceeds the HBM budget",
                  (unsigned long long)((size_t)s->N * s->W * 8));
    const int kind = s->manifold == CS_MANIFOLD_DESITTER ? kLinkDeSitter : s->d;
    const size_t wb = link_workspace_bytes(kind, s->N);
    if (wb) {
      s->link_work = ctx->pool.alloc(wb);
      if (!s->link_work) {
        ctx->pool.release(s->bits);
        s->bits = nullptr;
        return fail(CS_ENOMEM, "cs_link: link tables of %llu bytes exceed the HBM budget",
                    (unsigned long long)wb);
      }
    }
    hipError_t e = launch_link(kind, s->N, s->coords, s->bits, s->W, s->link_work, ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "link launch");
  }
  s->linked = true;
  s->counted_kmax = -1;
  return CS_OK;
}

static cs_status check_count_args(cs_ctx* ctx, cs_set* s, int kmax, int path) {
  if (!ctx || !s) return fail(CS_EINVAL, "NULL argument");
  if (kmax < 3 || kmax > CS_KMAX_MAX) return fail(CS_EINVAL, "kmax must be in [3, %d], got %d", CS_KMAX_MAX, kmax);
  if (path < CS_PATH_AUTO || path > CS_PATH_MFMA_FP4) return fail(CS_EINVAL, "bad path %d", path);
  if (path == CS_PATH_MFMA_FP4 && s->N >= (1 << 24))
    return fail(CS_EINVAL, "the FP4 path needs N < 2^24 (exact fp32 sums)");
  if (!s->linked) return fail(CS_EINVAL, "set is not linked");
  return CS_OK;
}

cs_status cs_interval_abundances(cs_ctx* ctx, cs_set* s, int kmax, uint64_t* out, uint64_t* R_out,
                                 uint64_t* summ_out, int path) {
  cs_status rc = check_count_args(ctx, s, kmax, path);
  if (rc != CS_OK) return rc;
  if (!out) return fail(CS_EINVAL, "cs_interval_abundances: out is NULL");
  (void)hipSetDevice(ctx->device);
  std::vector<uint64_t> tot((size_t)kmax + 3, 0);
  if (path == CS_PATH_AUTO && (s->d == 2 || s->d == 4)) path = tuned_path(ctx, s->d, s->N);
  if (path == CS_PATH_AUTO) path = choose_path(s->N, kmax);
  s->last_path = path;
  if (s->N > 1) {
    rc = count_matrix(ctx, s->bits, s->N, s->W, kmax, path, tot.data(), nullptr, ctx->stream);
    if (rc != CS_OK) return rc;
  }
  std::memcpy(out, tot.data(), (size_t)(kmax + 1) * 8);
  if (R_out) *R_out = tot[(size_t)kmax + 1];
  if (summ_out) *summ_out = tot[(size_t)kmax + 2];
  for (int k = 0; k < 4; ++k) s->n[k] = tot[(size_t)k];
  s->R = tot[(size_t)kmax + 1];
  s->summ = tot[(size_t)kmax + 2];
  s->counted_kmax = kmax;
  return CS_OK;
}

cs_status cs_interval_abundances_rows(cs_ctx* ctx, cs_set* s, int kmax, uint64_t* blocks, int path) {
  cs_status rc = check_count_args(ctx, s, kmax, path);
  if (rc != CS_OK) return rc;
  if (!blocks) return fail(CS_EINVAL, "cs_interval_abundances_rows: blocks is NULL");
  (void)hipSetDevice(ctx->device);
  const int64_t nrb = num_row_blocks(s->N);
  if (s->N <= 1) {
    std::memset(blocks, 0, (size_t)nrb * (kmax + 3) * 8);
    return CS_OK;
  }
  std::vector<uint64_t> tot((size_t)kmax + 3, 0);
  rc = count_matrix(ctx, s->bits, s->N, s->W, kmax, path, tot.data(), blocks, ctx->stream);
  if (rc != CS_OK) return rc;
  for (int k = 0; k < 4; ++k) s->n[k] = tot[(size_t)k];
  s->R = tot[(size_t)kmax + 1];
  s->summ = tot[(size_t)kmax + 2];
  s->counted_kmax = kmax;
  return CS_OK;
}

cs_status cs_bd_action(cs_ctx* ctx, cs_set* s, double* S_out) {
  if (!ctx || !s || !S_out) return fail(CS_EINVAL, "cs_bd_action: NULL argument");
  if (s->d != 2 && s->d != 4) return fail(CS_EINVAL, "cs_bd_action: set has no dimension (d=%d)", s->d);
  if (s->counted_kmax < 0) {
    uint64_t n[4];
    cs_status rc = cs_interval_abundances(ctx, s, 3, n, nullptr, nullptr, CS_PATH_AUTO);
    if (rc != CS_OK) return rc;
  }
  *S_out = bd_action(s->d, s->N, s->n);
  return CS_OK;
}

cs_status cs_smeared_action(cs_ctx* ctx, cs_set* s, double eps, double* S_out) {
  if (!ctx || !s || !S_out) return fail(CS_EINVAL, "cs_smeared_action: NULL argument");
  if (s->d != 2) return fail(CS_EINVAL, "cs_smeared_action: Eq. 5 is the 2D smeared action (set d=%d)", s->d);
  if (!(eps > 0.0 && eps <= 1.0)) return fail(CS_EINVAL, "cs_smeared_action: eps must be in (0, 1]");
  const int kmax = (int)std::max<int64_t>(s->N - 2, 3);
  std::vector<uint64_t> hist((size_t)kmax + 1);
  cs_status rc = cs_interval_abundances(ctx, s, kmax, hist.data(), nullptr, nullptr, CS_PATH_AUTO);
  if (rc != CS_OK) return rc;
  *S_out = smeared_action(s->N, hist.data(), (int64_t)hist.size(), eps);
  return CS_OK;
}

uint64_t cs_link_workspace_bytes(int d, int64_t N) {
  if ((d != 2 && d != 4) || N < 0) return 0;
  return (uint64_t)link_workspace_bytes(d, N);
}

cs_status cs_link_dev(int d, int64_t N, const double* coords_dev, uint64_t* bits_dev, int64_t stride_words,
                      void* work_dev, uint64_t work_bytes, void* hip_stream) {
  if (d != 2 && d != 4) return fail(CS_EINVAL, "cs_link_dev: d must be 2 or 4");
  if (N < 0) return fail(CS_EINVAL, "cs_link_dev: N < 0");
  if (N == 0) return CS_OK;
  if (!coords_dev || !bits_dev) return fail(CS_EINVAL, "cs_link_dev: NULL pointer");
  if (stride_words < row_words(N) || stride_words % 4)
    return fail(CS_EINVAL, "cs_link_dev: stride must be >= %lld and a multiple of 4", (long long)row_words(N));
  const uint64_t need = (uint64_t)link_workspace_bytes(d, N);
  if (need && (!work_dev || work_bytes < need))
    return fail(CS_EINVAL, "cs_link_dev: workspace of %llu bytes needed, %llu given", (unsigned long long)need,
                (unsigned long long)(work_dev ? work_bytes : 0));
  hipError_t e = launch_link(d, N, coords_dev, bits_dev, stride_words, work_dev, (hipStream_t)hip_stream);
  return e == hipSuccess ? CS_OK : hip_fail(e, "cs_link_dev");
}

uint64_t cs_count_workspace_bytes(int64_t N, int kmax) {
  if (N < 0 || kmax < 3) return 0;
  const int64_t nrb = num_row_blocks(N);
  return (uint64_t)((nrb > 0 ? nrb : 1) * (kmax + 3)) * 8;
}

cs_status cs_count_dev(const uint64_t* bits_dev, int64_t N, int64_t stride_words, int kmax, uint64_t* stats_dev,
                       void* work_dev, int path, void* hip_stream) {
  if (N < 0) return fail(CS_EINVAL, "cs_count_dev: N < 0");
  if (kmax < 3 || kmax > CS_KMAX_MAX) return fail(CS_EINVAL, "cs_count_dev: bad kmax %d", kmax);
  if (path < CS_PATH_AUTO || path > CS_PATH_MFMA_FP4) return fail(CS_EINVAL, "cs_count_dev: bad path");
  if (path == CS_PATH_MFMA_FP4 && N >= (1 << 24))
    return fail(CS_EINVAL, "cs_count_dev: the FP4 path needs N < 2^24");
  if (!stats_dev || !work_dev || (N > 0 && !bits_dev)) return fail(CS_EINVAL, "cs_count_dev: NULL pointer");
  if (N > 0 && (stride_words < row_words(N) || stride_words % 4))
    return fail(CS_EINVAL, "cs_count_dev: stride must be >= %lld and a multiple of 4", (long long)row_words(N));
  hipStream_t st = (hipStream_t)hip_stream;
  const int64_t nrb = num_row_blocks(N);
  const size_t nws = (size_t)(nrb > 0 ? nrb : 1) * (kmax + 3);
  hipError_t e = init_count_mfma();
  if (e == hipSuccess) e = launch_fill_u64((uint64_t*)work_dev, 0, nws, st);
  if (e == hipSuccess && N > 1) e = run_count(bits_dev, N, stride_words, kmax, path, (uint64_t*)work_dev, st);
  if (e == hipSuccess) e = launch_reduce_rows((uint64_t*)work_dev, nrb > 0 ? nrb : 1, kmax, stats_dev, st);
  return e == hipSuccess ? CS_OK : hip_fail(e, "cs_count_dev");
}


// ---- the count with a library-held workspace ----------------------------------
// A fixed device array stands in for the caller's workspace.  Its name in
// host code is not a device address: each device's copy is looked up once
// with hipGetSymbolAddress (with that device current) and only that pointer
// is handed to kernels.
namespace {
static __device__ __align__(256) uint64_t scratch[CS_COUNT_STATIC_WORDS];
std::mutex g_scratch_mu;
std::vector<void*> g_scratch_dev;  // per device id
}  // namespace

static cs_status scratch_for_current_device(uint64_t** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "cs_count_dev_static: hipGetDevice");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if ((size_t)dev >= g_scratch_dev.size()) g_scratch_dev.resize((size_t)dev + 1, nullptr);
  if (!g_scratch_dev[(size_t)dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e, "cs_count_dev_static: hipGetSymbolAddress");
    g_scratch_dev[(size_t)dev] = p;
  }
  *out = (uint64_t*)g_scratch_dev[(size_t)dev];
  return CS_OK;
}

cs_status cs_count_dev_static(const uint64_t* bits_dev, int64_t N, int64_t stride_words, int kmax,
                              uint64_t* stats_dev, int path, void* hip_stream) {
  if (N < 0) return fail(CS_EINVAL, "cs_count_dev_static: N < 0");
  if (kmax < 3 || kmax > CS_KMAX_MAX) return fail(CS_EINVAL, "cs_count_dev_static: bad kmax %d", kmax);
  if (path < CS_PATH_AUTO || path > CS_PATH_MFMA_FP4) return fail(CS_EINVAL, "cs_count_dev_static: bad path");
  if (path == CS_PATH_MFMA_FP4 && N >= (1 << 24))
    return fail(CS_EINVAL, "cs_count_dev_static: the FP4 path needs N < 2^24");
  if (!stats_dev || (N > 0 && !bits_dev)) return fail(CS_EINVAL, "cs_count_dev_static: NULL pointer");
  if (N > 0 && (stride_words < row_words(N) || stride_words % 4))
    return fail(CS_EINVAL, "cs_count_dev_static: stride must be >= %lld and a multiple of 4",
                (long long)row_words(N));
  const int64_t nrb = num_row_blocks(N);
  const uint64_t nws = (uint64_t)(nrb > 0 ? nrb : 1) * (uint64_t)(kmax + 3);
  if (nws > CS_COUNT_STATIC_WORDS)
    return fail(CS_EINVAL, "cs_count_dev_static: N=%lld with kmax=%d needs %llu workspace words, "
                "more than the library's %d", (long long)N, kmax, (unsigned long long)nws,
                CS_COUNT_STATIC_WORDS);
  uint64_t* ws = nullptr;
  cs_status rc = scratch_for_current_device(&ws);
  if (rc != CS_OK) return rc;
  hipStream_t st = (hipStream_t)hip_stream;
  hipError_t e = init_count_mfma();
  if (e == hipSuccess) e = launch_fill_u64(ws, 0, (size_t)nws, st);
  if (e == hipSuccess && N > 1) e = run_count(bits_dev, N, stride_words, kmax, path, ws, st);
  if (e == hipSuccess) e = launch_reduce_rows(ws, nrb > 0 ? nrb : 1, kmax, stats_dev, st);
  return e == hipSuccess ? CS_OK : hip_fail(e, "cs_count_dev_static");
}

// ---- local abundances by the saturating count -------------------------------

uint64_t cs_count_local_workspace_bytes(int64_t N) {
  if (N < 0) return 0;
  return sat_workspace_bytes(N);
}

cs_status cs_count_local_dev(const uint64_t* bits_dev, int64_t N, int64_t stride_words, uint64_t* stats_dev,
                             void* work_dev, uint64_t work_bytes, void* hip_stream) {
  if (N < 0) return fail(CS_EINVAL, "cs_count_local_dev: N < 0");
  if (!stats_dev || !work_dev || (N > 0 && !bits_dev)) return fail(CS_EINVAL, "cs_count_local_dev: NULL pointer");
  if (N > 0 && (stride_words < row_words(N) || stride_words % 4))
    return fail(CS_EINVAL, "cs_count_local_dev: stride must be >= %lld and a multiple of 4", (long long)row_words(N));
  if (work_bytes < sat_workspace_bytes(N))
    return fail(CS_EINVAL, "cs_count_local_dev: workspace must hold %llu bytes",
                (unsigned long long)sat_workspace_bytes(N));
  hipError_t e = launch_count_sat(bits_dev, N, stride_words, kSatChunk, kSatMargin, (uint64_t*)work_dev, stats_dev,
                                  (hipStream_t)hip_stream);
  return e == hipSuccess ? CS_OK : hip_fail(e, "cs_count_local_dev");
}

cs_status cs_local_abundances(cs_ctx* ctx, cs_set* s, uint64_t* out, uint64_t* blocks) {
  if (!ctx || !s || !out) return fail(CS_EINVAL, "cs_local_abundances: NULL argument");
  if (!s->linked) return fail(CS_EINVAL, "cs_local_abundances: set is not linked");
  (void)hipSetDevice(ctx->device);
  const int64_t N = s->N, nb = (N + 63) / 64;
  const uint64_t wb = sat_workspace_bytes(N);
  DevBuf work(ctx->pool, wb + 64);  // block slots, then the 6 totals
  if (!work.p) return fail(CS_ENOMEM, "cs_local_abundances: no room for %llu bytes of counters",
                           (unsigned long long)(wb + 64));
  uint64_t* stats = (uint64_t*)((char*)work.p + wb);
  hipError_t e = launch_count_sat(s->bits, N, s->W, kSatChunk, kSatMargin, (uint64_t*)work.p, stats, ctx->stream);
  uint64_t h[6] = {0, 0, 0, 0, 0, 0};
  std::vector<uint64_t> blk;
  if (e == hipSuccess) e = hipMemcpyAsync(h, stats, sizeof h, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess && blocks && nb > 0) {
    blk.resize((size_t)nb * kSatBlkWords);
    e = hipMemcpyAsync(blk.data(), work.p, blk.size() * 8, hipMemcpyDeviceToHost, ctx->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(e, "cs_local_abundances");
  std::memcpy(out, h, 6 * 8);
  if (blocks)
    for (int64_t b = 0; b < nb; ++b)
      for (int k = 0; k < 5; ++k) blocks[b * 5 + k] = blk[(size_t)b * kSatBlkWords + k];
  for (int k = 0; k < 4; ++k) s->n[k] = h[k];
  s->R = h[4];
  s->summ = 0;
  s->counted_kmax = 3;
  s->last_path = CS_PATH_LOCAL;
  return CS_OK;
}

}  // extern "C"
