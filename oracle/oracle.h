/*
 * oracle.h - plain, slow, single-threaded CPU oracle for the asynchronous block-I/O
 * path (AGILE, arXiv 2504.19365).
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the benchmark's CPU
 * baseline leg may load or call this code.  The product path never routes through it.
 * It shares no code with the GPU path; its only common dependency is the seeded input
 * generator module, which holds none of the method's arithmetic.
 *
 * The software cache and the NVMe-style queues are transparent to results (Sec. 3.4:
 * every access is routed through the cache only to coalesce requests and keep copies
 * coherent), so the oracle computes every workload result from its plain definition by
 * reading the store image directly.  A sequential clock-replacement simulator (the
 * policy of Sec. 4.4) gives the exact hit/miss/victim trace that a one-request-at-a-time
 * run of the cache must reproduce.
 *
 * Parity status: every function below is pinned by a CPU test against something other
 * than itself (closed forms, library routines, hand-worked traces, brute force); see
 * the test files named next to each function.
 */
#ifndef AGILE_ORACLE_H
#define AGILE_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* f_K(v): K iterations of v = fmaf(v, 0.999f, 0.001f).  The paper sweeps a per-element
 * compute loop to set the computation-to-communication ratio (Sec. 4.2); these constants
 * keep values O(1) and normal.  Pin: closed form 1 + 0.999^K (v - 1) (test_oracle_core). */
float oracle_fK(float v, uint32_t K);

/* Gather: out[i] = the row_bytes bytes of global row rows[i] of the image
 * (row r at byte offset r * row_bytes).  Pin: numpy view indexing (test_oracle_core). */
void oracle_gather(const uint8_t* image, uint64_t row_bytes, const int64_t* rows, uint64_t n,
                   uint8_t* out);

/* Embedding-bag forward over T concatenated fp32 tables of `rows` x `dim`.
 * Bag g = b*T + t covers lookups [off[g], off[g+1]) of table t = g % T.
 * out[g*dim + d] = sum over the bag's lookups, in order, of f_K(table_t[idx[j]][d]),
 * fp32 accumulator from +0.0f with plain fp32 adds.
 * bags == NULL computes all B*T bags; otherwise only the listed bag ids, writing
 * out[k*dim + d] for the k-th listed bag.
 * Pins: fp64 sums within Higham's recursive-summation bound, tiny numpy float32 loop
 * (test_oracle_core). */
void oracle_embbag_forward(const uint8_t* image, uint64_t rows, uint32_t dim, uint32_t T,
                           const int64_t* idx, const int64_t* off, uint64_t B, uint32_t K,
                           const int64_t* bags, uint64_t nbags, float* out);

/* The same forward with its bags spread over all cores (OpenMP), each bag computed by
 * oracle_embbag_forward: the all-cores CPU baseline (cpu_baseline.c).  Pin: equals
 * oracle_embbag_forward bit for bit (test_oracle_core). */
void oracle_embbag_forward_par(const uint8_t* image, uint64_t rows, uint32_t dim, uint32_t T,
                               const int64_t* idx, const int64_t* off, uint64_t B, uint32_t K,
                               float* out);
int oracle_par_threads(void);

/* Embedding-bag backward (K = 0) fused with SGD, in place on the image.
 * Loss L = sum_g sum_d grad_out[g][d] * pooled[g][d]; dL/dW_t[r][d] is the sum of
 * grad_out[g][d] over the occurrences (g, j) of row r of table t, taken in ascending
 * lookup position j (which is ascending (bag, position)) with an fp32 accumulator from
 * +0.0f; then W' = fmaf(-lr, grad, W).  Returns the number of distinct rows updated.
 * Pins: dense A^T g in fp64, central finite differences (test_oracle_core). */
uint64_t oracle_embbag_backward_sgd(uint8_t* image, uint64_t rows, uint32_t dim, uint32_t T,
                                    const int64_t* idx, const int64_t* off, uint64_t B,
                                    const float* grad_out, float lr);

/* Level-synchronous top-down BFS over out-edges of a CSR graph (Sec. 4.5 runs BFS
 * without application-level optimisation).  level[src] = 0, unreached = -1.
 * Pins: scipy shortest paths, Graph500-style validation (test_oracle_graph). */
void oracle_bfs(const int64_t* row_ptr, const int32_t* col, uint64_t V, int64_t src,
                int32_t* level);

/* Graph500-style BFS validation, independent of oracle_bfs.  Returns 0 when:
 * level[src] == 0; every edge (u, v) with u reached has v reached and
 * level[v] <= level[u] + 1; every reached v != src has an in-neighbour at level[v] - 1.
 * Otherwise returns the (1-based) number of the violated rule. */
int oracle_bfs_validate(const int64_t* row_ptr, const int32_t* col, uint64_t V, int64_t src,
                        const int32_t* level);

/* CSR SpMV: y[i] = fold over k ascending in row i of acc = fmaf(val[k], x[col[k]], acc),
 * acc from +0.0f.  rows [r0, r1) only.  Pins: scipy.sparse fp64 within bound, tiny
 * numpy float32 loop (test_oracle_graph). */
void oracle_spmv(const int64_t* row_ptr, const int32_t* col, const float* val, const float* x,
                 uint64_t r0, uint64_t r1, float* y);

/* Sequential set-associative cache with clock (second-chance) replacement.
 * set = line_id mod sets.  Each way: valid, tag, ref, dirty; one hand per set from 0.
 * access(line, write): hit -> ref = 1, dirty |= write.
 * miss -> starting at the hand: a way that is invalid or has ref == 0 is the victim;
 *         otherwise clear its ref and advance.  The hand then points past the victim.
 *         A dirty victim counts one write-back.  The fill sets ref = 1, dirty = write.
 * flush() writes back every dirty line once (set-major, way order), clears dirty and
 * keeps the lines valid.  Pin: hand-worked traces (tests/golden/clock_traces.txt). */
typedef struct oracle_clock oracle_clock;
oracle_clock* oracle_clock_new(uint32_t sets, uint32_t assoc);
void oracle_clock_free(oracle_clock* c);
/* Returns 1 on hit, 0 on miss; *way = the way hit or filled. */
int oracle_clock_access(oracle_clock* c, uint64_t line_id, int write, int32_t* way);
void oracle_clock_run(oracle_clock* c, const uint64_t* lines, const uint8_t* writes, uint64_t n,
                      uint8_t* hit, int32_t* way);
uint64_t oracle_clock_flush(oracle_clock* c);
/* counters[0..3] = hits, misses, write-backs on eviction, write-backs at flush */
void oracle_clock_counters(const oracle_clock* c, uint64_t* counters);
/* tags[s*assoc + w] = tag or -1 when invalid; dirty[...] = 0/1 */
void oracle_clock_state(const oracle_clock* c, int64_t* tags, uint8_t* dirty);

/* Ideal overlap speedup, Eq. 1 (Sec. 4.2): 1 + CTC for 0 <= CTC <= 1, 1 + 1/CTC above. */
double oracle_eq1(double ctc);

/* Interleaving over several devices (Sec. 4.3: request i goes to device i mod n), one
 * unit of unit_bytes at a time.  Unit u of the logical image is unit u / n of device
 * u mod n.  split: logical (units * unit_bytes bytes, units a multiple of n) ->
 * devs[d] (units / n units each).  Pins: a hand-worked 3-device example, n = 1 is the
 * identity, and every unit lands once (test_oracle_stripe). */
void oracle_stripe_split(const uint8_t* logical, uint64_t units, uint64_t unit_bytes, uint32_t n,
                         uint8_t* const* devs);

/* Writes of whole units in the given order (a later write of a unit replaces an earlier
 * one): unit lines[i] of image takes src + i * unit_bytes.  The write of Sec. 3.5's
 * API as seen in the store once it is done.  Pins: hand-worked overwrite order and
 * untouched units unchanged (test_oracle_stripe). */
void oracle_write_units(uint8_t* image, uint64_t unit_bytes, const uint64_t* lines, uint64_t k,
                        const uint8_t* src);

#ifdef __cplusplus
}
#endif
#endif
