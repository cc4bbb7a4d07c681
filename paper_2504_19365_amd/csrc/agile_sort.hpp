// agile_sort.hpp - device-wide exclusive scan and stable LSD radix sort for gfx950.
//
// Two building blocks of the write path and the graph workloads: the backward pass sorts
// the (row << 32 | lookup position) keys of a batch by row so that every distinct row's
// occurrences sit together in ascending position (Sec. 3.4 case d, the read-modify-write
// of a row happens once per batch), and each BFS level turns its frontier's out-degrees
// into edge offsets with an exclusive prefix sum (Sec. 4.5).
//
// Both work on tiles of TILE = 4096 elements per 1024-thread workgroup (4 per thread,
// consecutive), use wave64 cross-lane operations inside a wave and LDS across the 16
// waves of a workgroup, and are deterministic (no atomics decide an order).
//   * Scan: reduce each tile, scan the tile sums (recursively when there are more than one
//     tile of them), then scan every tile again from its offset.
//   * Sort: per pass of DIGIT_BITS bits, a digit histogram per tile, one scan of the
//     digit-major histogram table (digit d of tile b at d * tiles + b, so the scan gives
//     every (digit, tile) its global start in stable order), and a scatter in which every
//     key's rank among equal digits follows input order: earlier rounds of the tile, then
//     earlier waves of the round, then earlier lanes of the wave.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ag {
namespace sort {

constexpr uint32_t BLOCK = 1024;
constexpr uint32_t ITEMS = 4;
constexpr uint32_t TILE = BLOCK * ITEMS;
constexpr uint32_t WAVES = BLOCK / 64;
constexpr uint32_t DIGIT_BITS = 8;
constexpr uint32_t DIGITS = 1u << DIGIT_BITS;

__host__ __device__ constexpr uint64_t tiles_of(uint64_t n) { return (n + TILE - 1) / TILE; }

// Inclusive scan across the 64 lanes of a wave (Hillis-Steele over lane shuffles).
template <class T>
__device__ __forceinline__ T wave_incl_scan(T v) {
  const uint32_t l = __lane_id();
#pragma unroll
  for (uint32_t o = 1; o < 64; o <<= 1) {
    const T u = __shfl_up(v, o, 64);
    if (l >= o) v += u;
  }
  return v;
}

// Exclusive scan of the values `v` of every thread of a 1024-thread workgroup, in thread
// order; returns the thread's exclusive prefix and writes the workgroup total to *total.
template <class T>
__device__ __forceinline__ T block_excl_scan(T v, T* total) {
  __shared__ T wsum[WAVES];
  const uint32_t w = threadIdx.x / 64;
  const T inc = wave_incl_scan(v);
  if (__lane_id() == 63) wsum[w] = inc;
  __syncthreads();
  if (threadIdx.x < 64) {
    T s = threadIdx.x < WAVES ? wsum[threadIdx.x] : T(0);
    const T si = wave_incl_scan(s);
    if (threadIdx.x < WAVES) wsum[threadIdx.x] = si - s;  // exclusive over waves
    if (threadIdx.x == WAVES - 1) *total = si;
  }
  __syncthreads();
  const T r = wsum[w] + inc - v;
  __syncthreads();  // wsum may be reused by the caller's next round
  return r;
}

// Tile sums: sums[b] = sum of in[b*TILE, min(n, (b+1)*TILE)).
template <class T>
__global__ __launch_bounds__(BLOCK) void k_scan_reduce(const T* in, uint64_t n, T* sums) {
  __shared__ T tot;
  const uint64_t base = (uint64_t)blockIdx.x * TILE + (uint64_t)threadIdx.x * ITEMS;
  T s = 0;
#pragma unroll
  for (uint32_t i = 0; i < ITEMS; ++i)
    if (base + i < n) s += in[base + i];
  block_excl_scan<T>(s, &tot);
  __syncthreads();
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// out[i] = offs[b] (0 when offs is NULL) + sum of in[tile start .. i) for i in tile b.
// In-place use (out == in) is allowed: every thread reads its items before any write.
template <class T>
__global__ __launch_bounds__(BLOCK) void k_scan_tile(const T* in, uint64_t n, const T* offs, T* out) {
  __shared__ T tot;
  const uint64_t base = (uint64_t)blockIdx.x * TILE + (uint64_t)threadIdx.x * ITEMS;
  T v[ITEMS];
  T s = 0;
#pragma unroll
  for (uint32_t i = 0; i < ITEMS; ++i) {
    v[i] = base + i < n ? in[base + i] : T(0);
    s += v[i];
  }
  T p = block_excl_scan<T>(s, &tot) + (offs ? offs[blockIdx.x] : T(0));
#pragma unroll
  for (uint32_t i = 0; i < ITEMS; ++i) {
    if (base + i < n) out[base + i] = p;
    p += v[i];
  }
}

// Work area (elements of T) an exclusive scan of n elements needs for its tile sums, all
// levels included.
__host__ __device__ constexpr uint64_t scan_work_elems(uint64_t n) {
  return n <= TILE ? 0 : tiles_of(n) + scan_work_elems(tiles_of(n));
}

// Exclusive scan of n elements of `in` into `out` (may alias) on `stream`; `work` holds
// scan_work_elems(n) elements.  Returns false when a launch failed.
template <class T>
bool exclusive_scan(const T* in, T* out, uint64_t n, T* work, hipStream_t stream) {
  if (n == 0) return true;
  const uint64_t nt = tiles_of(n);
  if (nt == 1) {
    hipLaunchKernelGGL(k_scan_tile<T>, dim3(1), dim3(BLOCK), 0, stream, in, n, (const T*)nullptr, out);
    return hipGetLastError() == hipSuccess;
  }
  T* sums = work;
  hipLaunchKernelGGL(k_scan_reduce<T>, dim3((uint32_t)nt), dim3(BLOCK), 0, stream, in, n, sums);
  if (hipGetLastError() != hipSuccess) return false;
  if (!exclusive_scan<T>(sums, sums, nt, work + nt, stream)) return false;
  hipLaunchKernelGGL(k_scan_tile<T>, dim3((uint32_t)nt), dim3(BLOCK), 0, stream, in, n, (const T*)sums, out);
  return hipGetLastError() == hipSuccess;
}

__device__ __forceinline__ uint32_t digit_of(uint64_t key, uint32_t shift, uint32_t mask) {
  return (uint32_t)(key >> shift) & mask;
}

// Digit histogram of tile b, digit-major: hist[d * tiles + b].
__global__ __launch_bounds__(BLOCK) void k_radix_hist(const uint64_t* keys, uint64_t n, uint32_t shift,
                                                      uint32_t mask, uint32_t* hist, uint32_t tiles) {
  __shared__ uint32_t h[DIGITS];
  for (uint32_t d = threadIdx.x; d < DIGITS; d += BLOCK) h[d] = 0;
  __syncthreads();
  const uint64_t base = (uint64_t)blockIdx.x * TILE;
#pragma unroll
  for (uint32_t i = 0; i < ITEMS; ++i) {
    const uint64_t p = base + (uint64_t)i * BLOCK + threadIdx.x;
    if (p < n) atomicAdd(&h[digit_of(keys[p], shift, mask)], 1u);
  }
  __syncthreads();
  for (uint32_t d = threadIdx.x; d < DIGITS; d += BLOCK) hist[(uint64_t)d * tiles + blockIdx.x] = h[d];
}

// Lanes of the wave whose digit equals this lane's (a match over the digit's bits).
__device__ __forceinline__ uint64_t digit_peers(uint32_t dg, bool act, uint32_t bits) {
  uint64_t m = __ballot(act);
  for (uint32_t b = 0; b < bits; ++b) {
    const uint64_t ones = __ballot(act && ((dg >> b) & 1u));
    m &= ((dg >> b) & 1u) ? ones : ~ones;
  }
  return m;
}

// Stable scatter of tile b: key p goes to out[start(d, b) + rank of p among the tile's
// keys with digit d, in input order], start = the scanned histogram table.  The tile is
// visited in ITEMS rounds of BLOCK consecutive keys (round i holds keys
// [base + i*BLOCK, base + (i+1)*BLOCK), wave w the 64 of them from w*64).
__global__ __launch_bounds__(BLOCK) void k_radix_scatter(const uint64_t* keys, uint64_t n, uint32_t shift,
                                                         uint32_t mask, uint32_t bits, const uint32_t* starts,
                                                         uint32_t tiles, uint64_t* out) {
  __shared__ uint32_t run[DIGITS];          // keys of each digit placed so far (all rounds)
  __shared__ uint32_t wcnt[WAVES][DIGITS];  // this round: keys of each digit per wave
  const uint32_t w = threadIdx.x / 64;
  for (uint32_t d = threadIdx.x; d < DIGITS; d += BLOCK) run[d] = starts[(uint64_t)d * tiles + blockIdx.x];
  const uint64_t base = (uint64_t)blockIdx.x * TILE;
  for (uint32_t i = 0; i < ITEMS; ++i) {
    for (uint32_t k = threadIdx.x; k < WAVES * DIGITS; k += BLOCK) (&wcnt[0][0])[k] = 0;
    __syncthreads();
    const uint64_t p = base + (uint64_t)i * BLOCK + threadIdx.x;
    const bool act = p < n;
    const uint64_t key = act ? keys[p] : 0;
    const uint32_t dg = act ? digit_of(key, shift, mask) : 0;
    const uint64_t peers = digit_peers(dg, act, bits);
    const uint32_t lane = __lane_id();
    const uint32_t below = (uint32_t)__popcll(peers & ((1ull << lane) - 1ull));
    // the lowest lane of each digit group records the group's size
    if (act && below == 0) wcnt[w][dg] = (uint32_t)__popcll(peers);
    __syncthreads();
    // per digit: exclusive prefix over the waves, added to the running start
    for (uint32_t d = threadIdx.x; d < DIGITS; d += BLOCK) {
      uint32_t s = run[d];
      for (uint32_t v = 0; v < WAVES; ++v) {
        const uint32_t c = wcnt[v][d];
        wcnt[v][d] = s;
        s += c;
      }
      run[d] = s;
    }
    __syncthreads();
    if (act) out[wcnt[w][dg] + below] = key;
    __syncthreads();
  }
}

// Work area of a radix sort of n keys: the alternate key buffer (n u64), the histogram
// table (DIGITS * tiles u32, scanned in place) and the scan's own work area.
__host__ __device__ constexpr uint64_t radix_work_bytes(uint64_t n) {
  return ((n * 8 + 255) / 256) * 256 + ((DIGITS * tiles_of(n) * 4 + 255) / 256) * 256 +
         ((scan_work_elems(DIGITS * tiles_of(n)) * 4 + 255) / 256) * 256;
}

// Stable LSD radix sort of n u64 keys by bits [lo, hi) (the other bits ride along):
// `keys` holds the input; on return *sorted points at `keys` or at the alternate buffer
// in `work` (radix_work_bytes(n) bytes), whichever holds the result.  Keys with equal
// sort bits keep their input order.  Returns false when a launch failed.
inline bool radix_sort(uint64_t* keys, uint64_t n, uint32_t lo, uint32_t hi, void* work, hipStream_t stream,
                       uint64_t** sorted) {
  *sorted = keys;
  if (n <= 1 || hi <= lo) return true;
  const uint64_t tiles = tiles_of(n);
  uint8_t* wb = (uint8_t*)work;
  uint64_t* alt = (uint64_t*)wb;
  uint32_t* hist = (uint32_t*)(wb + ((n * 8 + 255) / 256) * 256);
  uint32_t* swork = (uint32_t*)((uint8_t*)hist + ((DIGITS * tiles * 4 + 255) / 256) * 256);
  uint64_t* src = keys;
  uint64_t* dst = alt;
  for (uint32_t shift = lo; shift < hi; shift += DIGIT_BITS) {
    const uint32_t bits = (hi - shift) < DIGIT_BITS ? (hi - shift) : DIGIT_BITS;
    const uint32_t mask = (1u << bits) - 1u;
    hipLaunchKernelGGL(k_radix_hist, dim3((uint32_t)tiles), dim3(BLOCK), 0, stream, src, n, shift, mask, hist,
                       (uint32_t)tiles);
    if (hipGetLastError() != hipSuccess) return false;
    if (!exclusive_scan<uint32_t>(hist, hist, DIGITS * tiles, swork, stream)) return false;
    hipLaunchKernelGGL(k_radix_scatter, dim3((uint32_t)tiles), dim3(BLOCK), 0, stream, src, n, shift, mask, bits,
                       hist, (uint32_t)tiles, dst);
    if (hipGetLastError() != hipSuccess) return false;
    uint64_t* t = src;
    src = dst;
    dst = t;
  }
  *sorted = src;
  return true;
}

}  // namespace sort
}  // namespace ag
