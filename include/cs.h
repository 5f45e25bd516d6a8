/*
 * cs.h -- C ABI of the MI355X (gfx950) causal-set interval-abundance library.
 *
 * The library generates causal sets by sprinkling into flat causal diamonds,
 * links them into a packed adjacency matrix, counts the elements inside the
 * interval of every related pair, and evaluates the Benincasa-Dowker (BD)
 * action, after W. J. Cunningham and D. Krioukov, "Causal Set Generator and
 * Action Computer", arXiv:1709.03013.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Dimension d is the SPACETIME dimension: 2 = (1+1), 4 = (3+1).
 *  - Elements carry labels 0..N-1 in a topological (time) order: a related
 *    pair i<j always has i earlier (Sec. 2.2).
 *  - Coordinates are structure-of-arrays float64: d arrays of N doubles.
 *    2D: light-cone (u, v) in [0,1)^2, i<j related iff u_i<u_j and v_i<v_j.
 *    4D: (t, x, y, z) in the diamond |x| < min(t, 1-t), related iff
 *    dt*dt > (dx*dx + dy*dy) + dz*dz, evaluated in binary64 without fused
 *    multiply-add (Sec. 1.1: timelike separation, strict).
 *  - The causal matrix is symmetric with a zero diagonal (Sec. 2.2): row i
 *    has W = cs_row_words(N) uint64 words (ceil(N/64) rounded up to a
 *    multiple of 4, i.e. 256-bit rows, Sec. 3.2); column k is bit k%64 of
 *    word k/64 (LSB first); padding bits are zero.
 *  - Interval abundances: N_k = number of related pairs i<j with exactly k
 *    elements l, i<l<j, related to both (Sec. 4.1; Fig. 2 and Alg. 5 compute
 *    the same count as popcount(row i AND row j) over columns i+1..j-1).
 *    The paper's n_i (inclusive order interval i) is N_{i-1}.
 *  - Every call returns cs_status; nothing throws across the ABI.  On error
 *    cs_last_error() returns a thread-local message (valid until the next
 *    call on the same thread).  Results are bit-identical across paths, runs
 *    and batch compositions: all counting is in integers.
 *  - Thread safety: a context may be used from one thread at a time, except
 *    the queue calls (cs_queue_*), which may be called concurrently.
 */
#ifndef CS_H
#define CS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CS_OK = 0,
  CS_EINVAL = 1,        /* bad argument: d not 2/4, N<0, bad stride, kmax<3 ... */
  CS_ENOMEM = 2,        /* allocation would exceed the HBM budget, or failed */
  CS_EDEVICE = 3,       /* a HIP runtime error */
  CS_EBUSY = 4,         /* queue: result not ready yet */
  CS_EUNSUPPORTED = 5   /* not available on this device / build */
} cs_status;

enum {
  CS_PATH_AUTO = 0,     /* library picks the fastest path for the size (timed once) */
  CS_PATH_POP = 1,      /* VALU AND + popcount kernel */
  CS_PATH_MFMA = 2,     /* int8 MFMA contraction (future x past), int32 sums */
  CS_PATH_MFMA_FP4 = 3, /* the same contraction with FP4 (e2m1) 0/1 operands and
                           exact fp32 sums (m < 2^24); N must be below 2^24 */
  CS_PATH_LOCAL = 4     /* not a path of cs_interval_abundances: what
                           cs_set_count_path reports after cs_local_abundances */
};

typedef struct cs_ctx cs_ctx;
typedef struct cs_set cs_set;

/* Words per packed row for N elements: ceil(N/64) rounded up to 4. */
int64_t cs_row_words(int64_t N);

/* ---------------------------------------------------------------- context */
/* Create a context on HIP device `device`.  hbm_budget_bytes caps the device
 * memory the context may hold (0 = 90% of free memory at creation).
 * hip_stream: a hipStream_t to run on, or NULL for a library-owned stream.
 * The library owns the context; free with cs_destroy. */
cs_status cs_create(cs_ctx** out, int device, uint64_t hbm_budget_bytes,
                    void* hip_stream);
void cs_destroy(cs_ctx* ctx);
/* Thread-local message for the last failed call on this thread. */
const char* cs_last_error(void);
/* Bytes of device memory the context currently holds for live sets. */
uint64_t cs_bytes_in_use(const cs_ctx* ctx);

/* --------------------------------------------------------------- sprinkle */
/* Sprinkle N elements into the flat diamond of dimension d from `seed` and
 * sort them by time (Sec. 2.1, 2.2).  Random numbers: Philox4x64-10 at
 * counter (c,0,0,0), key (seed, 1) in 2D / (seed, 2) in 4D; a word r gives
 * the double (r>>11) 2^-53.  2D element c: u = dbl(r0), v = dbl(r1); sorted
 * by t = (u+v)/2 (exact), then u, then c.  4D candidate c: t = dbl(r0),
 * x,y,z = dbl(r1..r3) - 1/2, accepted iff (x*x+y*y)+z*z < m*m,
 * m = min(t, 1-t); the first N accepted, sorted by t then acceptance rank.
 * Creates a device-resident set (coordinates only; call cs_link next),
 * owned by the library until cs_set_free.  N = 0 and N = 1 are valid. */
cs_status cs_sprinkle(cs_ctx* ctx, int d, int64_t N, uint64_t seed,
                      cs_set** out);

/* Coordinate manifold of a set (cs_set_manifold). */
enum { CS_MANIFOLD_DIAMOND = 0, CS_MANIFOLD_DESITTER = 1 };

/* Sprinkle N elements into the (1+1) de Sitter slab of Sec. 6.1 (Eq. 9),
 * ds^2 = sec^2(eta)(-deta^2 + dtheta^2), eta in [-eta0, eta0], theta on the
 * circle, and sort them by time.  The volume element is dw dtheta with
 * w = tan(eta), so w is uniform on [-w0, w0], w0 = tan(eta0) (host libm).
 * Element c, attempt a = 0..63: Philox4x64-10 at counter (c, a, 0, 0), key
 * (seed, 5); w = (2 dbl(r0) - 1) w0, direction x = 2 dbl(r1) - 1,
 * y = 2 dbl(r2) - 1, accepted iff 0 < x*x + y*y < 1 (after 64 rejections
 * (x, y) = (1, 0); w is the last attempt's).  Sorted by w, then c.
 * Coordinates: 3 rows (w, x, y); (x, y) is the unnormalised direction of
 * theta.  The set has d = 2 (2D action weights); cs_link tests
 * |delta eta| > geodesic angle as dot > 0 and
 * |w_i - w_j| * dot > |cross| * (1 + w_i w_j).  0 < eta0 < pi/4 (the
 * tangent test needs |delta eta| < pi/2), else CS_EINVAL. */
cs_status cs_sprinkle_desitter(cs_ctx* ctx, int64_t N, uint64_t seed, double eta0,
                               cs_set** out);

/* Manifold (CS_MANIFOLD_*) of a set and its number of coordinate rows
 * (d for diamonds, 3 for de Sitter, 0 for a set imported as a matrix). */
cs_status cs_set_manifold(const cs_set* set, int* manifold, int* coord_rows);

/* Import coordinates (host, SoA, d*N doubles) already in a topological
 * order: the caller's order becomes the labels.  The buffer is copied. */
cs_status cs_set_from_coords(cs_ctx* ctx, int d, int64_t N,
                             const double* coords, cs_set** out);

/* Import a packed symmetric matrix (N rows of stride_words >= cs_row_words(N)
 * words; on_device != 0 means `rows` is a device pointer).  The rows are
 * copied into a W-word layout.  Labels must be a topological order of the
 * order the matrix encodes (Sec. 4.3: the method works on any such matrix).
 * validate != 0 checks symmetry, zero diagonal and zero padding on the
 * device and returns CS_EINVAL if any fails.  d (2, 4, or 0 for "none") only
 * selects the action weights. */
cs_status cs_set_from_bitset(cs_ctx* ctx, int d, int64_t N,
                             const uint64_t* rows, int64_t stride_words,
                             int on_device, int validate, cs_set** out);

void cs_set_free(cs_set* set);
cs_status cs_set_info(const cs_set* set, int* d, int64_t* N, int64_t* W,
                      int* linked);

/* Copy the sorted coordinates (rows*N doubles, SoA; rows from
 * cs_set_manifold) and, if orig != NULL, the
 * generation index of each sorted element, to host memory. */
cs_status cs_get_coords(cs_ctx* ctx, const cs_set* set, double* coords,
                        int64_t* orig);
/* Copy the packed matrix (N*W words) to host memory. */
cs_status cs_get_bitset(cs_ctx* ctx, const cs_set* set, uint64_t* rows);
/* Device pointer of the packed matrix (N*W words), NULL if not linked.
 * Valid until cs_set_free. */
const uint64_t* cs_set_bitset_dev(const cs_set* set);
/* Count path (CS_PATH_POP / MFMA / MFMA_FP4) used by the set's last
 * cs_interval_abundances call (what CS_PATH_AUTO resolved to); 0 if none. */
int cs_set_count_path(const cs_set* set);

/* ------------------------------------------------------------------- link */
/* Build the packed causal matrix from the set's coordinates (Sec. 2.2):
 * every pair tested, bits written in 64-bit words.  Allocates N*W*8 bytes
 * inside the set; CS_ENOMEM if that exceeds the budget. */
cs_status cs_link(cs_ctx* ctx, cs_set* set);

/* ------------------------------------------------------------- abundances */
/* Interval abundances of a linked set.  out[0..kmax] receives N_0..N_kmax
 * (host memory, caller-owned, kmax+1 entries, kmax >= 3); R_out the number
 * of related pairs, summ_out the sum of interior counts over related pairs
 * (either may be NULL).  path: CS_PATH_AUTO / POP / MFMA / MFMA_FP4; the
 * result does not depend on it.  kmax is at most CS_KMAX_MAX; kmax = N-2
 * gives the full histogram (bins beyond 8191 are added to device memory with
 * atomics, so very large kmax is slower than kmax = 3). */
#define CS_KMAX_MAX 16777213
cs_status cs_interval_abundances(cs_ctx* ctx, cs_set* set, int kmax,
                                 uint64_t* out, uint64_t* R_out,
                                 uint64_t* summ_out, int path);

/* As above, plus the per-row-block breakdown: rows are grouped in blocks of
 * CS_ROW_BLOCK labels; blocks[b*(kmax+3) + k] holds, for pairs i<j with i in
 * block b, N_k (k = 0..kmax), then R, then the sum of interior counts.
 * blocks is host memory of ceil(N/CS_ROW_BLOCK)*(kmax+3) words. */
#define CS_ROW_BLOCK 256
cs_status cs_interval_abundances_rows(cs_ctx* ctx, cs_set* set, int kmax,
                                      uint64_t* blocks, int path);

/* ------------------------------------------------------- local abundances */
/* N_0..N_3 and R only, by a saturating count: Eq. 4 and its 4D counterpart
 * use only the intervals with at most three elements (Sec. 1.2), so each
 * pair's count stops once it reaches 4.  Every pair with m <= 3 still gets
 * its exact m, so N_0..N_3 and R are identical to cs_interval_abundances'
 * (Sec. 4.1 definition); bins above 3 and the sum of interior counts are not
 * computed.  One workgroup per 64x64 tile of pairs counts a few words in the
 * middle of the pairs' label ranges (staged in LDS), which settles most
 * pairs, then continues the others, 16 lanes per pair, until they reach 4
 * or their words are exhausted.  out (host, 6 words): N_0..N_3, R, and the
 * number of pairs that had to be continued from HBM beyond the staged
 * window (a diagnostic).  blocks (host, nullable): ceil(N/64)*5 words, for
 * each block b of 64 labels N_0..N_3 and R of the pairs i<j with i in block
 * b.  Device memory: 64 bytes per block of 64 labels, from the context's
 * pool.  Afterwards cs_bd_action uses these counts and cs_set_count_path
 * reports CS_PATH_LOCAL.  The middle chunk is 8 words and the staged
 * margin on each side 4 words; the result does not depend on them. */
cs_status cs_local_abundances(cs_ctx* ctx, cs_set* set, uint64_t* out, uint64_t* blocks);

/* ----------------------------------------------------------------- action */
/* Benincasa-Dowker action of a counted (or countable) set, using the set's d:
 *   2D (Eq. 4):  S = 2 (N - 2 N_0 + 4 N_1 - 2 N_2)
 *   4D (weights of the BD reference the paper cites for Eq. 4):
 *                S = (4/sqrt 6) (N - N_0 + 9 N_1 - 16 N_2 + 8 N_3)
 * in units of the discreteness scale.  The bracket is an exact 64-bit
 * integer; the one multiplication by the prefactor is the only rounding.
 * Counts the set (path AUTO) if it has not been counted yet.  CS_EINVAL if
 * the set has d = 0. */
cs_status cs_bd_action(cs_ctx* ctx, cs_set* set, double* S_out);

/* Smeared (non-local) BD action S_eps of Eq. 5, a 2D quantity (set d = 2):
 *   S_eps = 2 eps [N - 2 eps sum_k N_k f2(k, eps)],
 *   f2(k, eps) = q^k - 2 eps k q^(k-1) + eps^2 (k(k-1)/2) q^(k-2), q = 1-eps
 * (Eq. 5's f2 with the division by 1-eps multiplied out, so eps = 1 gives
 * Eq. 4 exactly).  Counts the full histogram N_0..N_{N-2} exactly on the
 * device, then sums on the host in a fixed order: q^k by repeated
 * multiplication, k ascending.  0 < eps <= 1, else CS_EINVAL. */
cs_status cs_smeared_action(cs_ctx* ctx, cs_set* set, double eps, double* S_out);

/* ----------------------------------------------------- device-pointer tier */
/* The caller owns all memory and the stream; calls are asynchronous on
 * `hip_stream` (a hipStream_t; NULL = the legacy default stream).
 * coords_dev: d*N doubles (SoA, topologically sorted).  bits_dev: N rows of
 * stride_words (>= cs_row_words(N), multiple of 4) words.
 * The link (Sec. 2.2) of a flat diamond.  In 2D it needs device scratch of
 * cs_link_workspace_bytes(2, N) bytes (per block of 64 labels: its sorted
 * u and v values and prefix masks, 2112 bytes), in use until the link has
 * finished on hip_stream; in 4D the size is 0 and work_dev may be NULL.
 * CS_EINVAL for d not 2 or 4, N < 0, a bad stride, NULL pointers or a
 * workspace below the size; nothing is launched then. */
uint64_t cs_link_workspace_bytes(int d, int64_t N);
cs_status cs_link_dev(int d, int64_t N, const double* coords_dev,
                      uint64_t* bits_dev, int64_t stride_words,
                      void* work_dev, uint64_t work_bytes, void* hip_stream);
/* Count from a device matrix.  stats_dev receives kmax+3 uint64 words:
 * N_0..N_kmax, R, sum of interior counts (device memory, overwritten).
 * work_dev: device scratch of cs_count_workspace_bytes(N, kmax) bytes. */
uint64_t cs_count_workspace_bytes(int64_t N, int kmax);
cs_status cs_count_dev(const uint64_t* bits_dev, int64_t N,
                       int64_t stride_words, int kmax, uint64_t* stats_dev,
                       void* work_dev, int path, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the count
 * of cs_count_dev with its workspace in a fixed device array of the library
 * (CS_COUNT_STATIC_WORDS uint64 words, 1 MiB, held on every device the
 * library runs on until the process ends) instead of a caller's buffer.
 * Allocates nothing; the caller still owns bits_dev and stats_dev (kmax+3
 * words, overwritten).  CS_EINVAL if cs_count_workspace_bytes(N, kmax)
 * exceeds the array (e.g. N = 2^17 allows kmax <= 253), or for the
 * arguments cs_count_dev rejects.  path CS_PATH_AUTO uses the fixed size
 * threshold (no timing runs).  The array is cleared by a kernel at the start
 * of every call; calls that overlap on one device (other streams, other
 * threads) share it and race. */
#define CS_COUNT_STATIC_WORDS 131072
cs_status cs_count_dev_static(const uint64_t* bits_dev, int64_t N,
                              int64_t stride_words, int kmax, uint64_t* stats_dev,
                              int path, void* hip_stream);

/* Local abundances from a device matrix (the saturating count above).
 * stats_dev receives 6 uint64 words: N_0..N_3, R, pairs continued from HBM.
 * work_dev: device scratch of work_bytes >= cs_count_local_workspace_bytes(N)
 * bytes (64 per block of 64 labels; per-block counters, overwritten).
 * Asynchronous on hip_stream; CS_EINVAL for N < 0, a bad stride, NULL
 * pointers or a workspace below the size. */
uint64_t cs_count_local_workspace_bytes(int64_t N);
cs_status cs_count_local_dev(const uint64_t* bits_dev, int64_t N, int64_t stride_words,
                             uint64_t* stats_dev, void* work_dev, uint64_t work_bytes,
                             void* hip_stream);

/* ---------------------------------------------------------------- batched */
typedef struct {
  int32_t d;        /* 2 or 4 */
  int32_t reserved;
  int64_t N;        /* elements, 0 <= N <= CS_BATCH_NMAX */
  uint64_t seed;
} cs_req;

typedef struct {
  uint64_t n[4];    /* N_0..N_3 */
  uint64_t R;       /* related pairs */
  uint64_t summ;    /* sum of interior counts */
  double S;         /* BD action */
  int32_t status;   /* cs_status of this set */
  int32_t reserved;
} cs_result;

#define CS_BATCH_NMAX 16384
/* Run a whole ensemble (the Monte Carlo use of Sec. 1.2): every set is
 * sprinkled, sorted, linked, counted and its action evaluated, with all sets
 * sharing each launch; the counting is one persistent launch per count
 * kernel over the (set, tile) work items of every set, sorted longest first
 * and dealt to a fixed grid in snake order.  The launch sequence is captured
 * once per batch shape (the list of (d, N)) in a hipGraph and replayed.  The
 * first call of a shape also tunes it: for each (d, ceil(log2 N)) group not
 * seen before on the context, the popcount kernel and the matrix-core kernel
 * (fp4) with 128- and 256-row tiles are timed on that group's sets and the
 * fastest is kept (every candidate must give identical counts), then each
 * kernel's grid is timed; see cs_batch_last_info.  out[s] is the result of
 * reqs[s]; identical to running the set alone.  A request with d not 2 or 4
 * or N outside [0, CS_BATCH_NMAX] gets status CS_EINVAL in its own result.
 * Device memory comes from the context's pool (CS_ENOMEM if the batch does
 * not fit the budget). */
cs_status cs_batch_run(cs_ctx* ctx, int nsets, const cs_req* reqs,
                       cs_result* out);

/* What the batch tuner chose for the most recent cs_batch_run on the
 * context: the number of sets counted by each kernel (64-row popcount
 * tiles, 256- and 128-row matrix-core tiles), each kernel's persistent grid
 * (workgroups; 0 if unused), and the count kernels' time on that batch's
 * matrices with the first-guess choices and with the tuned ones (ms, best
 * of three, measured when the shape was first run). */
typedef struct {
  int32_t sets_pop, sets_mfma256, sets_mfma128;
  int32_t grid_pop, grid_mfma256, grid_mfma128;
  double count_ms_untuned, count_ms_tuned;
} cs_batch_info;
cs_status cs_batch_last_info(cs_ctx* ctx, cs_batch_info* out);

/* ---------------------------------------------------------- queued serving */
/* Continuous-batching request server on the context.  Requests are admitted
 * in arrival order while their footprint (matrix + coordinates + scratch)
 * fits under the budget and a slot is free; admitted requests run
 * concurrently on the slots' streams.  Matrices stay resident (LRU) under the
 * budget, keyed by (d, N, seed): a repeated request reuses its matrix.
 * cs_queue_start sets the number of slots (concurrent requests on the GPU)
 * and the budget for resident matrices (0 = the context budget). */
cs_status cs_queue_start(cs_ctx* ctx, int slots, uint64_t resident_budget);
cs_status cs_queue_submit(cs_ctx* ctx, const cs_req* req, uint64_t* ticket);
/* CS_OK with *out filled when done, CS_EBUSY if not yet, CS_EINVAL for an
 * unknown ticket.  timing (nullable, 3 doubles): submit->admit, admit->done,
 * submit->done in seconds. */
cs_status cs_queue_poll(cs_ctx* ctx, uint64_t ticket, cs_result* out,
                        double* timing);
/* The next finished request, in completion order, whatever its ticket:
 * waits up to timeout_s seconds (0 = do not wait) and returns CS_OK with
 * *ticket, *out and timing (nullable, as for cs_queue_poll) filled, or
 * CS_EBUSY if none finished in time.  A request is returned once, by either
 * call. */
cs_status cs_queue_next(cs_ctx* ctx, double timeout_s, uint64_t* ticket, cs_result* out,
                        double* timing);
/* Block until every submitted request is done. */
cs_status cs_queue_drain(cs_ctx* ctx);
/* Stop the server thread (also done by cs_destroy). */
cs_status cs_queue_stop(cs_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* CS_H */
