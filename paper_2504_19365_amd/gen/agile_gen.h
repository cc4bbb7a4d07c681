/*
 * agile_gen.h - seeded synthetic input generators.
 *
 * This module produces the inputs of every workload (embedding tables, Zipf lookup
 * indices, bag lengths, RMAT graphs in CSR form, dense vectors, upstream gradients,
 * request streams).  It holds none of the method's arithmetic: no cache, queue or
 * workload computation lives here.  Both the GPU path's tests/benchmarks and the CPU
 * oracle consume what it produces; it is the only code the two sides share.
 *
 * Random numbers come from one counter-based generator: the i-th output (0-based) of
 * SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number generators",
 * OOPSLA 2014) seeded with key(seed, stream) = seed XOR (stream << 56).  Any element can
 * therefore be regenerated on its own, in any order and on any number of threads, with
 * identical results.
 */
#ifndef AGILE_GEN_H
#define AGILE_GEN_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Stream identifiers: one per generated quantity. */
enum {
  GEN_S_VALUES = 1,   /* embedding table contents               */
  GEN_S_ZIPF = 2,     /* lookup indices                          */
  GEN_S_BAGLEN = 3,   /* bag lengths                             */
  GEN_S_RMAT = 4,     /* RMAT quadrant draws                     */
  GEN_S_RELABEL = 5,  /* RMAT vertex relabelling bijection       */
  GEN_S_X = 6,        /* dense SpMV operand                      */
  GEN_S_GRAD = 7,     /* upstream gradients                      */
  GEN_S_ARRIVAL = 8,  /* request inter-arrival times             */
  GEN_S_REQSIZE = 9,  /* request sizes                           */
  GEN_S_SRC = 10,     /* BFS source vertex                       */
  GEN_S_BLOCKS = 11,  /* uniform random block ids                */
  GEN_S_VAL = 12      /* CSR edge values                         */
};

/* i-th output of SplitMix64 seeded with key(seed, stream). */
uint64_t gen_u64(uint64_t seed, uint32_t stream, uint64_t i);
/* (h >> 11) * 2^-53, in [0, 1). */
double gen_u01(uint64_t seed, uint32_t stream, uint64_t i);

/* Table value rule: float(((h >> 40) * 2^-23) - 1), exactly representable, in [-1, 1).
 * Fills rows [row0, row0 + nrows) of a table of `dim` columns into dst (row-major,
 * dst points at row row0).  Multi-threaded; the result does not depend on threads. */
void gen_fill_table(float* dst, uint64_t row0, uint64_t nrows, uint32_t dim, uint64_t seed);

/* Bounded Zipf(alpha) over ranks 1..n: cum[k-1] = sum_{j<=k} j^-alpha, summed in
 * ascending j in fp64. */
void gen_zipf_cum(double* cum, uint64_t n, double alpha);
/* Draw: target = u * cum[n-1]; returns the first index i with cum[i] > target (the
 * 0-based rank), clamped to n-1.  Rank k maps to row k-1 (identity). */
int64_t gen_zipf_pick(const double* cum, uint64_t n, double u);
/* out[j] = zipf pick for draw number (i0 + j) of (seed, GEN_S_ZIPF). */
void gen_zipf_rows(const double* cum, uint64_t n, uint64_t seed, uint64_t i0, uint64_t count,
                   int64_t* out);

/* Uniform integers in [lo, hi]: lo + floor(u * (hi - lo + 1)), clamped to hi. */
void gen_uniform_int(uint64_t seed, uint32_t stream, uint64_t i0, uint64_t count, int64_t lo,
                     int64_t hi, int64_t* out);

/* Embedding-bag batch: B samples x T tables, bags in sample-major order
 * (bag id = b*T + t).  Bag lengths uniform in [len_lo, len_hi] (stream GEN_S_BAGLEN),
 * rows Zipf over each table's rows (stream GEN_S_ZIPF, draw number = global position).
 * offsets has B*T+1 entries; idx must hold offsets[B*T] entries (call with idx == NULL
 * first to get the total via the return value). */
uint64_t gen_embbag_batch(const double* cum, uint64_t rows, uint64_t B, uint32_t T,
                          uint32_t len_lo, uint32_t len_hi, uint64_t seed, int64_t* offsets,
                          int64_t* idx);

/* Uniform fp32 in [lo, hi): float(lo + (hi - lo) * u). */
void gen_uniform_f32(uint64_t seed, uint32_t stream, uint64_t count, double lo, double hi,
                     float* out);
/* Standard normal via Box-Muller on draws (2i, 2i+1), computed in fp64, cast to fp32. */
void gen_normal_f32(uint64_t seed, uint64_t count, float* out);

/* RMAT(a, b, c) graph with 2^scale vertices and edge_factor * 2^scale directed edges.
 * Edge e takes `scale` uniform draws (numbers e*scale + l of stream GEN_S_RMAT); level l
 * picks quadrant (0,0) if u < a, (0,1) if u < a+b, (1,0) if u < a+b+c, else (1,1),
 * building the source and destination from the most significant bit down.  Both
 * endpoints are then relabelled by the bijection v -> (v * m + k) mod 2^scale with m
 * odd, both derived from (seed, GEN_S_RELABEL).  Duplicates and self-loops are kept.
 * CSR rows are sorted by (src, dst).
 * Pass 1: gen_rmat_degrees fills deg[2^scale] (out-degrees).
 * Pass 2: gen_rmat_fill writes col[] given row_ptr (prefix sums of deg, int64, V+1
 *         entries) and sorts every row; if val != NULL also writes
 *         val[k] = float(u01(seed, GEN_S_VAL, k)), a function of the CSR position. */
void gen_rmat_degrees(uint32_t scale, uint32_t edge_factor, double a, double b, double c,
                      uint64_t seed, uint32_t* deg);
void gen_rmat_fill(uint32_t scale, uint32_t edge_factor, double a, double b, double c,
                   uint64_t seed, const int64_t* row_ptr, int32_t* col, float* val);
/* First draw i = 0, 1, ... of (seed, GEN_S_SRC) mod V whose out-degree is >= 1. */
int64_t gen_bfs_source(uint64_t seed, const int64_t* row_ptr, uint64_t V);

/* Uniform block ids in [0, nblocks). */
void gen_uniform_blocks(uint64_t seed, uint64_t count, uint64_t nblocks, int64_t* out);

/* Request stream: inter-arrival times exponential with mean 1/rate (seconds) and sizes
 * n = clamp(round(2^(max_log2 * u)), 1, 2^max_log2). */
void gen_requests(uint64_t seed, uint64_t count, double rate, uint32_t max_log2,
                  double* arrival_s, int64_t* size);

int gen_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
