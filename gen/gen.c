/*
 * Seeded synthetic column generator.
 *
 * This file produces INPUTS only: it holds none of the query arithmetic
 * (no hashing of keys, no predicates, no joins or sums).  Both the GPU path
 * and the CPU oracle are fed from it.
 *
 * Random source: splitmix64 (Vigna, public domain) used as a counter-based
 * generator, i.e. draw i of stream `seed` is mix(seed + (i + 1) * golden).
 * Because a draw depends only on (seed, i), any row range of a column can be
 * generated independently and in parallel, and a chunk [off, off + n) equals
 * the same rows of the whole column.
 *
 * Range reduction: Lemire's multiply-shift, floor(x * range / 2^64).
 * Permutations: Fisher-Yates with draws taken from the stream in order.
 * Zipf: inverse CDF by binary search over cumulative weights r^-s.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SM64_GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t sm64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* Draw number i (0-based) of the splitmix64 stream seeded with `seed`. */
static inline uint64_t sm64_at(uint64_t seed, uint64_t i) {
  return sm64_mix(seed + (i + 1) * SM64_GAMMA);
}

/* Lemire range reduction: uniform in [0, range) for range <= 2^64 - 1. */
static inline uint64_t bounded(uint64_t x, uint64_t range) {
  return (uint64_t)(((unsigned __int128)x * range) >> 64);
}

/* Uniform double in [0, 1) from the top 53 bits. */
static inline double unit53(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }

uint64_t gen_draw(uint64_t seed, uint64_t i) { return sm64_at(seed, i); }

void gen_uniform_i32(int32_t *out, int64_t n, int64_t lo, int64_t hi, uint64_t seed,
                     int64_t offset) {
  const uint64_t range = (uint64_t)(hi - lo) + 1u;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i)
    out[i] = (int32_t)(lo + (int64_t)bounded(sm64_at(seed, (uint64_t)(offset + i)), range));
}

void gen_uniform_i64(int64_t *out, int64_t n, int64_t lo, int64_t hi, uint64_t seed,
                     int64_t offset) {
  const uint64_t range = (uint64_t)(hi - lo) + 1u;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i)
    out[i] = lo + (int64_t)bounded(sm64_at(seed, (uint64_t)(offset + i)), range);
}

/* out = a uniformly shuffled permutation of base, base+1, ..., base+n-1. */
void gen_perm_i32(int32_t *out, int64_t n, int64_t base, uint64_t seed) {
  for (int64_t i = 0; i < n; ++i) out[i] = (int32_t)(base + i);
  uint64_t draw = 0;
  for (int64_t i = n - 1; i >= 1; --i) {
    int64_t j = (int64_t)bounded(sm64_at(seed, draw++), (uint64_t)i + 1u);
    int32_t t = out[i];
    out[i] = out[j];
    out[j] = t;
  }
}

/*
 * Zipf over ranks 1..nkeys with P(r) proportional to r^-s (s = 0 is uniform).
 * Rank r is emitted as the value r.
 */
int gen_zipf_i32(int32_t *out, int64_t n, int64_t nkeys, double s, uint64_t seed,
                 int64_t offset) {
  if (nkeys <= 0) return -1;
  if (s == 0.0) {
    gen_uniform_i32(out, n, 1, nkeys, seed, offset);
    return 0;
  }
  double *cdf = (double *)malloc((size_t)nkeys * sizeof(double));
  if (!cdf) return -1;
  double acc = 0.0;
  for (int64_t r = 1; r <= nkeys; ++r) {
    acc += pow((double)r, -s);
    cdf[r - 1] = acc;
  }
  const double total = acc;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    const double u = unit53(sm64_at(seed, (uint64_t)(offset + i))) * total;
    int64_t lo = 0, hi = nkeys - 1; /* smallest index with cdf[idx] > u */
    while (lo < hi) {
      int64_t mid = lo + (hi - lo) / 2;
      if (cdf[mid] > u) hi = mid; else lo = mid + 1;
    }
    out[i] = (int32_t)(lo + 1);
  }
  free(cdf);
  return 0;
}

/* Sizes log-uniform in [lo, hi]: round(lo * (hi/lo)^u). */
void gen_loguniform_i64(int64_t *out, int64_t n, double lo, double hi, uint64_t seed) {
  const double lr = log(hi / lo);
  for (int64_t i = 0; i < n; ++i) {
    double v = lo * exp(lr * unit53(sm64_at(seed, (uint64_t)i)));
    out[i] = (int64_t)llround(v);
  }
}

/* Poisson process: n arrival times (seconds) with rate lambda per second. */
void gen_poisson_arrivals(double *out, int64_t n, double lambda, uint64_t seed) {
  double t = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    t += -log1p(-unit53(sm64_at(seed, (uint64_t)i))) / lambda;
    out[i] = t;
  }
}
