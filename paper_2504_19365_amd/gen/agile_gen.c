/*
 * agile_gen.c - seeded synthetic input generators (see agile_gen.h).
 * Built with gcc -O2 -fopenmp; no workload arithmetic lives here.
 */
#include "agile_gen.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static inline uint64_t key_of(uint64_t seed, uint32_t stream) {
  return seed ^ ((uint64_t)stream << 56);
}

static inline uint64_t at(uint64_t key, uint64_t i) { return mix64(key + (i + 1) * GOLDEN); }

static inline double u01_of(uint64_t h) { return (double)(h >> 11) * 0x1.0p-53; }

uint64_t gen_u64(uint64_t seed, uint32_t stream, uint64_t i) {
  return at(key_of(seed, stream), i);
}

double gen_u01(uint64_t seed, uint32_t stream, uint64_t i) {
  return u01_of(at(key_of(seed, stream), i));
}

int gen_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void gen_fill_table(float* dst, uint64_t row0, uint64_t nrows, uint32_t dim, uint64_t seed) {
  const uint64_t key = key_of(seed, GEN_S_VALUES);
  const int64_t n = (int64_t)(nrows * dim);
  const uint64_t base = row0 * dim;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < n; ++e) {
    uint64_t h = at(key, base + (uint64_t)e);
    dst[e] = (float)((double)(h >> 40) * 0x1.0p-23 - 1.0);
  }
}

void gen_zipf_cum(double* cum, uint64_t n, double alpha) {
  double s = 0.0;
  for (uint64_t k = 1; k <= n; ++k) {
    s += pow((double)k, -alpha);
    cum[k - 1] = s;
  }
}

int64_t gen_zipf_pick(const double* cum, uint64_t n, double u) {
  const double target = u * cum[n - 1];
  uint64_t lo = 0, hi = n; /* first i in [lo, hi) with cum[i] > target */
  while (lo < hi) {
    uint64_t mid = lo + (hi - lo) / 2;
    if (cum[mid] > target)
      hi = mid;
    else
      lo = mid + 1;
  }
  if (lo >= n) lo = n - 1;
  return (int64_t)lo;
}

void gen_zipf_rows(const double* cum, uint64_t n, uint64_t seed, uint64_t i0, uint64_t count,
                   int64_t* out) {
  const uint64_t key = key_of(seed, GEN_S_ZIPF);
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < (int64_t)count; ++j)
    out[j] = gen_zipf_pick(cum, n, u01_of(at(key, i0 + (uint64_t)j)));
}

void gen_uniform_int(uint64_t seed, uint32_t stream, uint64_t i0, uint64_t count, int64_t lo,
                     int64_t hi, int64_t* out) {
  const uint64_t key = key_of(seed, stream);
  const double span = (double)(hi - lo + 1);
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < (int64_t)count; ++j) {
    int64_t v = lo + (int64_t)floor(u01_of(at(key, i0 + (uint64_t)j)) * span);
    out[j] = v > hi ? hi : v;
  }
}

uint64_t gen_embbag_batch(const double* cum, uint64_t rows, uint64_t B, uint32_t T,
                          uint32_t len_lo, uint32_t len_hi, uint64_t seed, int64_t* offsets,
                          int64_t* idx) {
  const uint64_t nb = B * T;
  const uint64_t klen = key_of(seed, GEN_S_BAGLEN);
  const double span = (double)(len_hi - len_lo + 1);
  uint64_t total = 0;
  for (uint64_t g = 0; g < nb; ++g) {
    if (offsets) offsets[g] = (int64_t)total;
    int64_t len = (int64_t)len_lo + (int64_t)floor(u01_of(at(klen, g)) * span);
    if (len > (int64_t)len_hi) len = len_hi;
    total += (uint64_t)len;
  }
  if (offsets) offsets[nb] = (int64_t)total;
  if (idx) gen_zipf_rows(cum, rows, seed, 0, total, idx);
  return total;
}

void gen_uniform_f32(uint64_t seed, uint32_t stream, uint64_t count, double lo, double hi,
                     float* out) {
  const uint64_t key = key_of(seed, stream);
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < (int64_t)count; ++j)
    out[j] = (float)(lo + (hi - lo) * u01_of(at(key, (uint64_t)j)));
}

void gen_normal_f32(uint64_t seed, uint64_t count, float* out) {
  const uint64_t key = key_of(seed, GEN_S_GRAD);
  const double two_pi = 6.283185307179586476925286766559;
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < (int64_t)count; ++j) {
    double u1 = ((double)(at(key, 2 * (uint64_t)j) >> 11) + 1.0) * 0x1.0p-53; /* (0, 1] */
    double u2 = u01_of(at(key, 2 * (uint64_t)j + 1));
    out[j] = (float)(sqrt(-2.0 * log(u1)) * cos(two_pi * u2));
  }
}

/* ---- RMAT ---------------------------------------------------------------------------- */

static inline void rmat_edge(uint64_t key, uint32_t scale, double a, double ab, double abc,
                             uint64_t e, uint64_t* src, uint64_t* dst) {
  uint64_t s = 0, d = 0;
  for (uint32_t l = 0; l < scale; ++l) {
    double u = u01_of(at(key, e * scale + l));
    uint64_t sb, db;
    if (u < a) {
      sb = 0; db = 0;
    } else if (u < ab) {
      sb = 0; db = 1;
    } else if (u < abc) {
      sb = 1; db = 0;
    } else {
      sb = 1; db = 1;
    }
    s = (s << 1) | sb;
    d = (d << 1) | db;
  }
  *src = s;
  *dst = d;
}

static inline void relabel_params(uint64_t seed, uint32_t scale, uint64_t* m, uint64_t* k) {
  const uint64_t mask = (scale >= 64) ? ~0ULL : ((1ULL << scale) - 1);
  *m = (gen_u64(seed, GEN_S_RELABEL, 0) | 1ULL) & mask;
  if (*m == 0) *m = 1;
  *k = gen_u64(seed, GEN_S_RELABEL, 1) & mask;
}

void gen_rmat_degrees(uint32_t scale, uint32_t edge_factor, double a, double b, double c,
                      uint64_t seed, uint32_t* deg) {
  const uint64_t V = 1ULL << scale, E = V * edge_factor, mask = V - 1;
  const uint64_t key = key_of(seed, GEN_S_RMAT);
  uint64_t m, k;
  relabel_params(seed, scale, &m, &k);
  memset(deg, 0, V * sizeof(uint32_t));
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < (int64_t)E; ++e) {
    uint64_t s, d;
    rmat_edge(key, scale, a, a + b, a + b + c, (uint64_t)e, &s, &d);
    s = (s * m + k) & mask;
    __atomic_fetch_add(&deg[s], 1u, __ATOMIC_RELAXED);
  }
}

static int cmp_i32(const void* x, const void* y) {
  int32_t a = *(const int32_t*)x, b = *(const int32_t*)y;
  return (a > b) - (a < b);
}

void gen_rmat_fill(uint32_t scale, uint32_t edge_factor, double a, double b, double c,
                   uint64_t seed, const int64_t* row_ptr, int32_t* col, float* val) {
  const uint64_t V = 1ULL << scale, E = V * edge_factor, mask = V - 1;
  const uint64_t key = key_of(seed, GEN_S_RMAT);
  uint64_t m, k;
  relabel_params(seed, scale, &m, &k);
  int64_t* cursor = (int64_t*)malloc(V * sizeof(int64_t));
  memcpy(cursor, row_ptr, V * sizeof(int64_t));
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < (int64_t)E; ++e) {
    uint64_t s, d;
    rmat_edge(key, scale, a, a + b, a + b + c, (uint64_t)e, &s, &d);
    s = (s * m + k) & mask;
    d = (d * m + k) & mask;
    int64_t pos = __atomic_fetch_add(&cursor[s], 1, __ATOMIC_RELAXED);
    col[pos] = (int32_t)d;
  }
  free(cursor);
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t v = 0; v < (int64_t)V; ++v) {
    int64_t n = row_ptr[v + 1] - row_ptr[v];
    if (n > 1) qsort(col + row_ptr[v], (size_t)n, sizeof(int32_t), cmp_i32);
  }
  if (val) {
    const uint64_t kv = key_of(seed, GEN_S_VAL);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < (int64_t)E; ++e) val[e] = (float)u01_of(at(kv, (uint64_t)e));
  }
}

int64_t gen_bfs_source(uint64_t seed, const int64_t* row_ptr, uint64_t V) {
  for (uint64_t i = 0; i < 1000000; ++i) {
    uint64_t v = gen_u64(seed, GEN_S_SRC, i) % V;
    if (row_ptr[v + 1] > row_ptr[v]) return (int64_t)v;
  }
  return -1;
}

void gen_uniform_blocks(uint64_t seed, uint64_t count, uint64_t nblocks, int64_t* out) {
  const uint64_t key = key_of(seed, GEN_S_BLOCKS);
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < (int64_t)count; ++j) out[j] = (int64_t)(at(key, (uint64_t)j) % nblocks);
}

void gen_requests(uint64_t seed, uint64_t count, double rate, uint32_t max_log2,
                  double* arrival_s, int64_t* size) {
  const uint64_t ka = key_of(seed, GEN_S_ARRIVAL), ks = key_of(seed, GEN_S_REQSIZE);
  double t = 0.0;
  const int64_t cap = (int64_t)1 << max_log2;
  for (uint64_t i = 0; i < count; ++i) {
    t += -log(1.0 - u01_of(at(ka, i))) / rate;
    arrival_s[i] = t;
    int64_t n = (int64_t)llround(pow(2.0, (double)max_log2 * u01_of(at(ks, i))));
    size[i] = n < 1 ? 1 : (n > cap ? cap : n);
  }
}
