/*
 * cpu_baseline.c - the all-cores variant of the CPU baseline.
 *
 * TEST INFRASTRUCTURE, like the rest of this directory: only the benchmark's CPU-baseline
 * leg calls it.  It runs the oracle's own embedding-bag loop (oracle_embbag_forward, one
 * bag per call) under an OpenMP parallel-for over the bags of a batch, reading the store
 * image directly from host memory with no cache simulation.  Every bag is computed by the
 * same single-threaded code in the same order, so the output equals the oracle's bit for
 * bit; only the bags are spread over the cores.
 */
#include <omp.h>

#include "oracle.h"

int oracle_par_threads(void) { return omp_get_max_threads(); }

void oracle_embbag_forward_par(const uint8_t* image, uint64_t rows, uint32_t dim, uint32_t T,
                               const int64_t* idx, const int64_t* off, uint64_t B, uint32_t K,
                               float* out) {
  const int64_t n = (int64_t)(B * T);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t g = 0; g < n; ++g)
    oracle_embbag_forward(image, rows, dim, T, idx, off, B, K, &g, 1, out + (uint64_t)g * dim);
}
