/*
 * Seeded synthetic column generator.
 *
 * This module only draws random numbers and lays them out as columns. It
 * holds none of the query pipeline's arithmetic (no filters, joins, hashing
 * or aggregation) and is the single input source shared by the CPU oracle and
 * the GPU library: both receive the arrays written here.
 *
 * Random stream: SplitMix64 (Steele, Lea, Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014; constants as published by
 * Vigna). Value i of stream (seed, stream) is the SplitMix64 output at
 * counter position i of a generator whose state starts at
 * splitmix64(seed ^ splitmix64(stream)). Being counter based, any slice of a
 * column can be regenerated on its own and threads split work freely.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t fmix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static inline uint64_t stream_key(uint64_t seed, uint64_t stream) {
  return fmix(seed ^ fmix(stream + GAMMA));
}

/* value at counter position i */
static inline uint64_t draw(uint64_t key, uint64_t i) {
  return fmix(key + (i + 1) * GAMMA);
}

/* Lemire multiply-shift range reduction of the high 32 bits into [0, range) */
static inline uint64_t below(uint64_t r, uint64_t range) {
  if (range <= 0xFFFFFFFFULL) return ((r >> 32) * range) >> 32;
  return r % range;
}

/* uniform double in [0,1) from 53 random bits */
static inline double unit(uint64_t r) { return (double)(r >> 11) * (1.0 / 9007199254740992.0); }

uint64_t hg_splitmix64(uint64_t x) { return fmix(x + GAMMA); }

uint64_t hg_draw(uint64_t seed, uint64_t stream, uint64_t i) {
  return draw(stream_key(seed, stream), i);
}

/* uniform integers in [lo, hi) (hi > lo), written as int8/int32/int64 by width */
#define UNIFORM_BODY(T)                                                   \
  uint64_t key = stream_key(seed, stream);                                \
  uint64_t range = (uint64_t)(hi - lo);                                   \
  _Pragma("omp parallel for schedule(static)")                            \
  for (int64_t i = 0; i < n; ++i)                                         \
    out[i] = (T)(lo + (int64_t)below(draw(key, (uint64_t)(offset + i)), range));

void hg_uniform_i8(uint64_t seed, uint64_t stream, int64_t offset, int64_t n,
                   int64_t lo, int64_t hi, int8_t* out) { UNIFORM_BODY(int8_t) }
void hg_uniform_i32(uint64_t seed, uint64_t stream, int64_t offset, int64_t n,
                    int64_t lo, int64_t hi, int32_t* out) { UNIFORM_BODY(int32_t) }
void hg_uniform_i64(uint64_t seed, uint64_t stream, int64_t offset, int64_t n,
                    int64_t lo, int64_t hi, int64_t* out) { UNIFORM_BODY(int64_t) }

/* categorical int8 column: value v with probability probs[v] (k <= 16) */
void hg_categorical_i8(uint64_t seed, uint64_t stream, int64_t offset, int64_t n,
                       const double* probs, int32_t k, int8_t* out) {
  double cum[16];
  double acc = 0.0;
  for (int j = 0; j < k && j < 16; ++j) { acc += probs[j]; cum[j] = acc; }
  for (int j = 0; j < k && j < 16; ++j) cum[j] /= acc;
  uint64_t key = stream_key(seed, stream);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double u = unit(draw(key, (uint64_t)(offset + i)));
    int v = 0;
    while (v < k - 1 && u >= cum[v]) ++v;
    out[i] = (int8_t)v;
  }
}

/*
 * Bijective scramble of 32-bit values ("lowbias32" integer hash published by
 * C. Wellons; every step is invertible), keyed by xor with a seed word.
 * Used to turn dense ranks/ids into sparse int32 keys without collisions.
 */
static inline uint32_t scramble32(uint32_t x, uint32_t k) {
  x ^= k;
  x ^= x >> 16; x *= 0x7feb352dU;
  x ^= x >> 15; x *= 0x846ca68bU;
  x ^= x >> 16;
  return x;
}

uint32_t hg_scramble32(uint32_t x, uint32_t k) { return scramble32(x, k); }

/* out[i] = scramble(first + i): distinct sparse int32 keys */
void hg_sparse_keys_i32(uint64_t seed, uint64_t stream, int64_t first, int64_t n, int32_t* out) {
  uint32_t k = (uint32_t)stream_key(seed, stream);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) out[i] = (int32_t)scramble32((uint32_t)(first + i), k);
}

/* foreign keys: uniform index into [0, ndim) mapped through the same scramble
   as hg_sparse_keys_i32(seed, key_stream, 0, ndim) so every value is a real key */
void hg_foreign_keys_i32(uint64_t seed, uint64_t stream, uint64_t key_stream, int64_t offset,
                         int64_t n, int64_t ndim, int32_t* out) {
  uint64_t key = stream_key(seed, stream);
  uint32_t k = (uint32_t)stream_key(seed, key_stream);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    uint64_t idx = below(draw(key, (uint64_t)(offset + i)), (uint64_t)ndim);
    out[i] = (int32_t)scramble32((uint32_t)idx, k);
  }
}

/*
 * Zipf-distributed keys: rank r in [1, nranks] with P(r) proportional to
 * r^-s, sampled by inverse CDF (binary search over the cumulative weights),
 * then scrambled into int32 keys. When scramble is 0 the rank itself is
 * written.
 */
void hg_zipf_i32(uint64_t seed, uint64_t stream, int64_t offset, int64_t n, int64_t nranks,
                 double s, int32_t scramble, int32_t* out) {
  double* cdf = (double*)malloc(sizeof(double) * (size_t)nranks);
  if (!cdf) return;
  double acc = 0.0;
  for (int64_t r = 0; r < nranks; ++r) { acc += pow((double)(r + 1), -s); cdf[r] = acc; }
  for (int64_t r = 0; r < nranks; ++r) cdf[r] /= acc;
  uint64_t key = stream_key(seed, stream);
  uint32_t k = (uint32_t)stream_key(seed, stream ^ 0x5A5A5A5AULL);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double u = unit(draw(key, (uint64_t)(offset + i)));
    int64_t lo = 0, hi = nranks - 1;
    while (lo < hi) {
      int64_t mid = (lo + hi) >> 1;
      if (cdf[mid] > u) hi = mid; else lo = mid + 1;
    }
    uint32_t rank = (uint32_t)(lo + 1);
    out[i] = scramble ? (int32_t)scramble32(rank, k) : (int32_t)rank;
  }
  free(cdf);
}

/* uniform doubles in [0,1) (used for workload-mix parameters, never for columns) */
void hg_unit_f64(uint64_t seed, uint64_t stream, int64_t offset, int64_t n, double* out) {
  uint64_t key = stream_key(seed, stream);
  for (int64_t i = 0; i < n; ++i) out[i] = unit(draw(key, (uint64_t)(offset + i)));
}
