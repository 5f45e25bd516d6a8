/*
 * cs_oracle.c -- CPU oracle for the causal-set interval-abundance path.
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the tests, the smoke check and
 * the CPU-baseline leg of the benchmark may load this library.  It shares no
 * code, header or constant table with the GPU library: everything here is
 * written again from the paper's definitions and from the published
 * definition of the Philox generator.
 *
 * Paper: W. J. Cunningham and D. Krioukov, "Causal Set Generator and Action
 * Computer", arXiv:1709.03013.
 *
 * What is computed, and where the paper defines it:
 *   - sprinkling: i.i.d. coordinates in a bounded region (Sec. 2.1, the
 *     Poisson process of Sec. 1.1 conditioned on N);
 *   - topological (time) order of the labels (Sec. 2.2);
 *   - the relation: timelike separation in flat space (Sec. 1.1);
 *   - the symmetric, zero-diagonal adjacency matrix packed into 64-bit
 *     blocks with zero padding to 256 bits (Sec. 2.2 and Sec. 3.2);
 *   - the interval abundances: for every related pair i<j the number of
 *     elements k with i<k<j related to both (Sec. 4.1, the naive triple loop;
 *     Fig. 2 and Alg. 5 compute the same number as a masked AND + popcount);
 *   - the Benincasa-Dowker action, Eq. 4 in 2D, and the 4D weights of the
 *     paper's cited BD reference (a reading, see the design notes).
 *
 * Readings where the paper is silent (RNG, sort tie-break, region, 4D
 * weights) are fixed below and listed in the repository's design notes.
 *
 * Plain C99 + OpenMP, compiled with -ffp-contract=off so that every double
 * operation is rounded once, in the order written.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11, "Parallel random       */
/* numbers: as easy as 1, 2, 3").  Ten rounds; each round multiplies words  */
/* 0 and 2 of the counter by the two Philox multipliers, swaps the halves   */
/* and xors in the key; the key is bumped by the two Weyl constants between */
/* rounds.                                                                  */
/* ------------------------------------------------------------------------ */
void orc_philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2],
                       uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
  uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint64_t k0 = key_in[0], k1 = key_in[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    unsigned __int128 p0 = (unsigned __int128)M0 * c0;
    unsigned __int128 p1 = (unsigned __int128)M1 * c2;
    uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    uint64_t n0 = hi1 ^ c1 ^ k0;
    uint64_t n1 = lo1;
    uint64_t n2 = hi0 ^ c3 ^ k1;
    uint64_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* A 64-bit random word becomes the double (r >> 11) * 2^-53 in [0,1). */
static double unit_double(uint64_t r) { return (double)(r >> 11) * 0x1.0p-53; }

/* Stream tags of the key's second word: 1 = 2D coordinates, 2 = 4D
 * candidates. */
#define TAG_2D 1ULL
#define TAG_4D 2ULL

/* ------------------------------------------------------------------------ */
/* Sprinkling and time sort (Sec. 2.1, 2.2).                                */
/* ------------------------------------------------------------------------ */
typedef struct {
  uint64_t k1, k2; /* primary and secondary time keys */
  int64_t idx;     /* generation index: the final tie-break */
} orc_key;

static int key_cmp(const void* pa, const void* pb) {
  const orc_key* a = (const orc_key*)pa;
  const orc_key* b = (const orc_key*)pb;
  if (a->k1 != b->k1) return a->k1 < b->k1 ? -1 : 1;
  if (a->k2 != b->k2) return a->k2 < b->k2 ? -1 : 1;
  if (a->idx != b->idx) return a->idx < b->idx ? -1 : 1;
  return 0;
}

/*
 * 2D diamond in light-cone coordinates: element c draws Philox at
 * counter (c,0,0,0), key (seed, 1); u = dbl(r0), v = dbl(r1).  With
 * u = a 2^-53 and v = b 2^-53 the time t = (u+v)/2 is (a+b) 2^-54 exactly,
 * so the sort key is the integer a+b, ties broken by a, then by c.
 *
 * 4D diamond of height 1: candidate c draws Philox at counter (c,0,0,0),
 * key (seed, 2); t = dbl(r0), x,y,z = dbl(r1..r3) - 0.5; it is accepted iff
 * (x*x + y*y) + z*z < m*m with m = min(t, 1-t).  The first N accepted
 * candidates, in candidate order, are the elements; element e (0-based
 * acceptance rank) is sorted by t = (r0 >> 11) 2^-53, ties broken by e.
 *
 * coords: d arrays of N doubles (SoA), written in sorted order.
 * orig:   (nullable) generation index of each sorted element.
 * Returns the number of candidates drawn (N in 2D), or -1 on bad input.
 */
int64_t orc_sprinkle(int d, int64_t N, uint64_t seed, double* coords,
                     int64_t* orig) {
  if (N < 0 || (d != 2 && d != 4)) return -1;
  if (N == 0) return 0;
  orc_key* keys = (orc_key*)malloc((size_t)N * sizeof(orc_key));
  double* raw = (double*)malloc((size_t)N * (size_t)d * sizeof(double));
  int64_t drawn = 0;
  if (d == 2) {
    const uint64_t key[2] = {seed, TAG_2D};
    for (int64_t c = 0; c < N; ++c) {
      uint64_t ctr[4] = {(uint64_t)c, 0, 0, 0}, r[4];
      orc_philox4x64_10(ctr, key, r);
      uint64_t a = r[0] >> 11, b = r[1] >> 11;
      raw[c] = unit_double(r[0]);
      raw[N + c] = unit_double(r[1]);
      keys[c].k1 = a + b;
      keys[c].k2 = a;
      keys[c].idx = c;
    }
    drawn = N;
  } else {
    const uint64_t key[2] = {seed, TAG_4D};
    int64_t e = 0;
    uint64_t c = 0;
    while (e < N) {
      uint64_t ctr[4] = {c, 0, 0, 0}, r[4];
      orc_philox4x64_10(ctr, key, r);
      double t = unit_double(r[0]);
      double x = unit_double(r[1]) - 0.5;
      double y = unit_double(r[2]) - 0.5;
      double z = unit_double(r[3]) - 0.5;
      double m = t < 1.0 - t ? t : 1.0 - t;
      double rho2 = (x * x + y * y) + z * z;
      if (rho2 < m * m) {
        raw[e] = t;
        raw[N + e] = x;
        raw[2 * N + e] = y;
        raw[3 * N + e] = z;
        keys[e].k1 = r[0] >> 11;
        keys[e].k2 = 0;
        keys[e].idx = e;
        ++e;
      }
      ++c;
    }
    drawn = (int64_t)c;
  }
  qsort(keys, (size_t)N, sizeof(orc_key), key_cmp);
  for (int64_t s = 0; s < N; ++s) {
    int64_t g = keys[s].idx;
    for (int q = 0; q < d; ++q) coords[(int64_t)q * N + s] = raw[(int64_t)q * N + g];
    if (orig) orig[s] = g;
  }
  free(keys);
  free(raw);
  return drawn;
}

/* ------------------------------------------------------------------------ */
/* The relation (Sec. 1.1): timelike separation, strict.                    */
/* coords are SoA, sorted; requires i < j.                                  */
/* ------------------------------------------------------------------------ */
int orc_related(int d, const double* coords, int64_t N, int64_t i, int64_t j) {
  if (d == 2) {
    const double* u = coords;
    const double* v = coords + N;
    return u[i] < u[j] && v[i] < v[j];
  }
  const double* t = coords;
  const double* x = coords + N;
  const double* y = coords + 2 * N;
  const double* z = coords + 3 * N;
  double dt = t[j] - t[i];
  double dx = x[j] - x[i];
  double dy = y[j] - y[i];
  double dz = z[j] - z[i];
  double s2 = (dx * dx + dy * dy) + dz * dz;
  return dt > 0.0 && dt * dt > s2;
}

/* Words per bitset row: ceil(N/64) rounded up to a multiple of 4, so every
 * row is 256-bit aligned with zero padding (Sec. 3.2). */
int64_t orc_row_words(int64_t N) {
  int64_t w = (N + 63) / 64;
  return (w + 3) / 4 * 4;
}

/* The adjacency matrix (Sec. 2.2): symmetric, zero diagonal; bit k of row i
 * lives in word k/64 at bit position k%64.  bits has N*W words. */
void orc_link(int d, const double* coords, int64_t N, uint64_t* bits,
              int64_t W) {
  memset(bits, 0, (size_t)N * (size_t)W * sizeof(uint64_t));
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < N; ++i) {
    uint64_t* row = bits + i * W;
    for (int64_t k = 0; k < N; ++k) {
      if (k == i) continue;
      int64_t lo = i < k ? i : k, hi = i < k ? k : i;
      if (orc_related(d, coords, N, lo, hi))
        row[k >> 6] |= 1ULL << (k & 63);
    }
  }
}

static int bit_at(const uint64_t* bits, int64_t W, int64_t i, int64_t k) {
  return (int)((bits[i * W + (k >> 6)] >> (k & 63)) & 1ULL);
}

/* ------------------------------------------------------------------------ */
/* Interval abundances, tier 1: the naive triple loop of Sec. 4.1 on the     */
/* coordinates (no bitset).  hist has nbins entries; m >= nbins is counted   */
/* only in R and summ.  Pairs i<j over rows [i_lo, i_hi).                    */
/* ------------------------------------------------------------------------ */
void orc_count_coords(int d, const double* coords, int64_t N, int64_t i_lo,
                      int64_t i_hi, int64_t nbins, uint64_t* hist,
                      uint64_t* R_out, uint64_t* summ_out) {
  memset(hist, 0, (size_t)nbins * sizeof(uint64_t));
  uint64_t R = 0, summ = 0;
  for (int64_t i = i_lo; i < i_hi; ++i) {
    for (int64_t j = i + 1; j < N; ++j) {
      if (!orc_related(d, coords, N, i, j)) continue;
      uint64_t m = 0;
      for (int64_t k = i + 1; k < j; ++k)
        if (orc_related(d, coords, N, i, k) && orc_related(d, coords, N, k, j))
          ++m;
      ++R;
      summ += m;
      if ((int64_t)m < nbins) ++hist[m];
    }
  }
  *R_out = R;
  *summ_out = summ;
}

/* Number of elements strictly between i and j related to both, read from
 * the bitset: the masked AND + popcount of Fig. 2, over bit positions
 * i+1 .. j-1 only.  Requires i < j. */
uint64_t orc_interval_size(const uint64_t* bits, int64_t W, int64_t i,
                           int64_t j) {
  const uint64_t* a = bits + i * W;
  const uint64_t* b = bits + j * W;
  uint64_t m = 0;
  int64_t lo = i + 1, hi = j - 1; /* inclusive bit range */
  if (lo > hi) return 0;
  int64_t wlo = lo >> 6, whi = hi >> 6;
  for (int64_t w = wlo; w <= whi; ++w) {
    uint64_t x = a[w] & b[w];
    if (w == wlo) x &= ~0ULL << (lo & 63);              /* bits >= lo */
    if (w == whi && (hi & 63) != 63) x &= (1ULL << ((hi & 63) + 1)) - 1; /* bits <= hi */
    m += (uint64_t)__builtin_popcountll(x);
  }
  return m;
}

/* Interval abundances, tier 2: every related pair i<j with i in
 * [i_lo, i_hi), m from orc_interval_size.  hist has nbins entries; m >= nbins
 * counts only in R and summ.  Threads keep private histograms that are
 * summed at the end (the reduction of Sec. 4.2). */
void orc_count_bits(const uint64_t* bits, int64_t N, int64_t W, int64_t i_lo,
                    int64_t i_hi, int64_t nbins, uint64_t* hist,
                    uint64_t* R_out, uint64_t* summ_out, int nthreads) {
  memset(hist, 0, (size_t)nbins * sizeof(uint64_t));
  uint64_t R = 0, summ = 0;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
#pragma omp parallel
  {
    uint64_t* h = (uint64_t*)calloc((size_t)nbins, sizeof(uint64_t));
    uint64_t r = 0, s = 0;
#pragma omp for schedule(dynamic, 1)
    for (int64_t i = i_lo; i < i_hi; ++i) {
      for (int64_t j = i + 1; j < N; ++j) {
        if (!bit_at(bits, W, i, j)) continue;
        uint64_t m = orc_interval_size(bits, W, i, j);
        ++r;
        s += m;
        if ((int64_t)m < nbins) ++h[m];
      }
    }
#pragma omp critical
    {
      for (int64_t b = 0; b < nbins; ++b) hist[b] += h[b];
      R += r;
      summ += s;
    }
    free(h);
  }
  *R_out = R;
  *summ_out = summ;
}

/* ------------------------------------------------------------------------ */
/* (1+1) de Sitter slab (Sec. 6.1, Eq. 9): ds^2 = sec^2(eta)(-deta^2 +       */
/* dtheta^2), eta in [-eta0, eta0], theta in [0, 2 pi).  The volume element  */
/* sec^2(eta) deta dtheta = dw dtheta with w = tan(eta), so elements are     */
/* uniform in w in [-w0, w0], w0 = tan(eta0), and in theta.  theta is kept   */
/* as an unnormalised direction (x, y) drawn uniformly from the unit disk:   */
/* only differences of angles enter, and tan of a difference is cross/dot.   */
/* Element c, attempt a = 0, 1, ..., 63: Philox at counter (c, a, 0, 0), key */
/* (seed, 5): w = (2 dbl(r0) - 1) w0, x = 2 dbl(r1) - 1, y = 2 dbl(r2) - 1,  */
/* accepted iff 0 < x*x + y*y < 1 (after 64 rejections (x, y) = (1, 0)).     */
/* Labels sorted by w, then c.  coords: 3 arrays (w, x, y).                 */
/* ------------------------------------------------------------------------ */
#define TAG_DS 5ULL

typedef struct {
  double w;
  int64_t idx;
} orc_wkey;

static int wkey_cmp(const void* pa, const void* pb) {
  const orc_wkey* a = (const orc_wkey*)pa;
  const orc_wkey* b = (const orc_wkey*)pb;
  if (a->w != b->w) return a->w < b->w ? -1 : 1;
  if (a->idx != b->idx) return a->idx < b->idx ? -1 : 1;
  return 0;
}

int64_t orc_sprinkle_desitter(int64_t N, uint64_t seed, double w0, double* coords,
                              int64_t* orig) {
  if (N < 0) return -1;
  if (N == 0) return 0;
  const uint64_t key[2] = {seed, TAG_DS};
  orc_wkey* keys = (orc_wkey*)malloc((size_t)N * sizeof(orc_wkey));
  double* raw = (double*)malloc((size_t)N * 3 * sizeof(double));
  int64_t draws = 0;
  for (int64_t c = 0; c < N; ++c) {
    double w = 0.0, x = 1.0, y = 0.0;
    for (uint64_t a = 0; a < 64; ++a) {
      uint64_t ctr[4] = {(uint64_t)c, a, 0, 0}, r[4];
      orc_philox4x64_10(ctr, key, r);
      ++draws;
      const double wc = (2.0 * unit_double(r[0]) - 1.0) * w0;
      const double xc = 2.0 * unit_double(r[1]) - 1.0;
      const double yc = 2.0 * unit_double(r[2]) - 1.0;
      const double rr = xc * xc + yc * yc;
      w = wc;
      if (rr > 0.0 && rr < 1.0) {
        x = xc;
        y = yc;
        break;
      }
      x = 1.0;
      y = 0.0;
    }
    raw[c] = w;
    raw[N + c] = x;
    raw[2 * N + c] = y;
    keys[c].w = w;
    keys[c].idx = c;
  }
  qsort(keys, (size_t)N, sizeof(orc_wkey), wkey_cmp);
  for (int64_t s = 0; s < N; ++s) {
    const int64_t g = keys[s].idx;
    for (int q = 0; q < 3; ++q) coords[(int64_t)q * N + s] = raw[(int64_t)q * N + g];
    if (orig) orig[s] = g;
  }
  free(keys);
  free(raw);
  return draws;
}

/* de Sitter relation (strict): |deta| > pi - |pi - |dtheta||.  For eta0 <
 * pi/4 both sides are below pi/2 when dot > 0, and tan is increasing there:
 * tan|deta| = |wi - wj| / (1 + wi wj), tan(dtheta) = |cross| / dot, so the
 * test is dot > 0 and |wi - wj| * dot > |cross| * (1 + wi wj). */
int orc_related_desitter(const double* coords, int64_t N, int64_t i, int64_t j) {
  const double* w = coords;
  const double* x = coords + N;
  const double* y = coords + 2 * N;
  const double dot = x[i] * x[j] + y[i] * y[j];
  const double cr = fabs(x[i] * y[j] - y[i] * x[j]);
  const double dw = fabs(w[i] - w[j]);
  const double b = 1.0 + w[i] * w[j];
  return dot > 0.0 && dw * dot > cr * b;
}

void orc_link_desitter(const double* coords, int64_t N, uint64_t* bits, int64_t W) {
  memset(bits, 0, (size_t)N * (size_t)W * sizeof(uint64_t));
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < N; ++i) {
    uint64_t* row = bits + i * W;
    for (int64_t k = 0; k < N; ++k) {
      if (k == i) continue;
      if (orc_related_desitter(coords, N, i < k ? i : k, i < k ? k : i))
        row[k >> 6] |= 1ULL << (k & 63);
    }
  }
}

/* Number of chains i < k < j with i~k and k~j, counted through the middle
 * element: sum over k of (#related below k) * (#related above k).  For a
 * transitive relation this equals the sum of m over related pairs. */
uint64_t orc_three_chains(const uint64_t* bits, int64_t N, int64_t W) {
  uint64_t tot = 0;
#pragma omp parallel for reduction(+ : tot) schedule(static)
  for (int64_t k = 0; k < N; ++k) {
    const uint64_t* row = bits + k * W;
    uint64_t below = 0, above = 0;
    for (int64_t w = 0; w < W; ++w) {
      uint64_t x = row[w];
      int64_t base = w * 64;
      uint64_t lowmask;
      if (base + 64 <= k) lowmask = ~0ULL;
      else if (base >= k) lowmask = 0;
      else lowmask = (1ULL << (k - base)) - 1;
      below += (uint64_t)__builtin_popcountll(x & lowmask);
      above += (uint64_t)__builtin_popcountll(x & ~lowmask);
    }
    tot += below * above;
  }
  return tot;
}

/* Benincasa-Dowker action from the abundances n[k] = #related pairs with
 * exactly k interior elements (k = 0..3).
 *   2D, Eq. 4:  S = 2 (N - 2 n0 + 4 n1 - 2 n2)
 *   4D (weights of the cited BD reference):
 *               S = (4/sqrt 6) (N - n0 + 9 n1 - 16 n2 + 8 n3)
 * The bracket is formed exactly in 64-bit integers; the product with the
 * prefactor is the only rounding.  Returns NAN for other d. */
double orc_bd_action(int d, int64_t N, const uint64_t* n) {
  if (d == 2) {
    int64_t K = N - 2 * (int64_t)n[0] + 4 * (int64_t)n[1] - 2 * (int64_t)n[2];
    return 2.0 * (double)K;
  }
  if (d == 4) {
    int64_t K = N - (int64_t)n[0] + 9 * (int64_t)n[1] - 16 * (int64_t)n[2] +
                8 * (int64_t)n[3];
    double c = 4.0 / sqrt(6.0);
    return c * (double)K;
  }
  return NAN;
}

/* Smeared BD action, Eq. 5 (2D):
 *   S_eps = 2 eps [ N - 2 eps sum_{i=1}^{N-1} n_i f2(i-1, eps) ]
 *   f2(k, eps) = (1-eps)^k [1 - 2 eps k/(1-eps) + eps^2 k(k-1) / (2 (1-eps)^2)]
 * with n_i = N_{i-1} (hist[k] = N_k, k = 0..nbins-1).  f2 is evaluated in the
 * algebraically equal form without division,
 *   f2(k) = q^k - 2 eps k q^(k-1) + eps^2 (k(k-1)/2) q^(k-2),  q = 1 - eps,
 * which is defined at eps = 1 (where Eq. 5 reduces to Eq. 4).  Evaluation
 * order (a reading the paper leaves open): q^k by repeated multiplication
 * from q^0 = 1; terms in the order written; the sum over k ascending. */
double orc_smeared_action(int64_t N, const uint64_t* hist, int64_t nbins, double eps) {
  const double q = 1.0 - eps;
  double pk = 1.0, pk1 = 0.0, pk2 = 0.0; /* q^k, q^(k-1), q^(k-2) */
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

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
