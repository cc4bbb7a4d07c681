// agile.hip - kernels and host implementation of the C ABI in include/agile.h.
//
// Every launch that can submit commands carries its own service wavefronts: workgroups
// [0, service_blocks) run the emulated controller and the completion service, the rest
// run user wavefronts.  Workgroups are dispatched in index order, and the user grid is
// sized to the resident capacity, so the service is always resident while users wait.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "agile.h"
#include "agile_dev.hpp"
#include "agile_sort.hpp"

using namespace ag;

// =============================================================================== kernels
namespace {

constexpr uint32_t TK_OK = 0, TK_EAGAIN = 1;

struct embbag_args {
  const int64_t* idx;
  const int64_t* off;   // NULL in gather mode (bag g = lookups [64g, 64g+64))
  float* out;
  uint64_t nbags;
  uint64_t n;           // lookups (gather mode)
  uint64_t rows;        // rows per table
  uint64_t base_off;    // byte offset of table 0 in the store
  uint64_t table_bytes;
  uint32_t T, dim, row_bytes, K;
  uint32_t mode, gather, active_waves, serve;
  // continuous batching (serve != 0): an unbounded stream of bags from requests that the
  // host publishes over time, held in rings: bag b in slot b & bag_mask, lookup j (a
  // position in the stream of lookups) in slot j & look_mask, request r in slot
  // r & req_mask.  idx and out are rings too.  The waves read HBM copies of the host's
  // rings, which the session's staging wave fills before it publishes; out and done
  // live in pinned host memory.
  const uint64_t* bag_j0;     // lookups [bag_j0, bag_j1) of the bag
  const uint64_t* bag_j1;
  const uint64_t* bag_req;    // request of the bag
  const uint32_t* bag_tab;    // table of the bag
  const uint32_t* req_nbags;  // bags of the request
  uint32_t* req_cnt;          // bags finished per request slot (device; the request's last
                              // bag returns its slot to zero)
  uint32_t* done;             // done[r & req_mask] = 1 once the request's outputs are visible
  const uint64_t* pub_dev;    // device mirror: [0] bags published, [1] stop
  const uint64_t* pub_host;   // pinned: [0] bags published, [1] stop
  uint64_t bag_mask, look_mask, req_mask;
  // the resident-hit launch before this one defers bags to this list, and this launch
  // runs only them; their number is the device counter C_DEFER, read by every wave when
  // it starts.  NULL: this launch runs every bag.
  const uint32_t* list;
};

// Per-wave state of the bag source.  Bags [0, 2A) of a launch with A active waves are
// dealt out statically (wave u starts with bags u and u + A); the rest are taken
// dynamically from P = min(WORK_PARTS, A) partitions (bag b in partition (b - 2A) mod P,
// each with its own counter): a wave starts at partition u mod P and moves on
// once its partition is used up, so no wave starts behind thousands of same-address
// atomics and the last bags still go to whichever waves are free.  The wave holds the next bag it
// will work on, taken (and its lookup range loaded) as soon as the previous one was
// taken, so that the atomic and the offset loads travel while the current bag is
// processed (except near the end of the launch).  A held bag whose request is not yet
// published stays held.  The work counters start every launch at zero.
struct src_state {
  int64_t g;       // position of the held bag in the launch's bag sequence, or -1
  int64_t bag;     // the held bag itself (differs from g when the launch runs a list)
  int64_t j0, j1;  // its lookups [j0, j1)
  bool exhausted;
  uint32_t uw;     // this wave's index among the active waves
  uint32_t dealt;  // static bags looked at so far (0..STATIC_ROUNDS)
  uint32_t tried;  // partitions found used up so far
  int64_t nb;      // bags of the launch: a.nbags, or the deferred count for a list
  int64_t A;       // waves taking part: a.active_waves, or fewer for a short list
};
constexpr uint32_t STATIC_ROUNDS = 2;

__device__ __forceinline__ float fK(float v, uint32_t K) {
  for (uint32_t k = 0; k < K; ++k) v = __builtin_fmaf(v, 0.999f, 0.001f);
  return v;
}

// Descriptor of one chunk: bag g, lookups [j, j + n), last chunk of its bag?
struct desc_t {
  int64_t g;
  int64_t j, end;
  uint32_t n;
  bool valid, last;
};

// A ring entry in pinned host memory, read at system scope: the host rewrites a slot
// for every lap of the ring, so no cached copy of an older lap may be used.
template <typename T>
__device__ __forceinline__ T ring_ld(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

template <int VPL>
__device__ __forceinline__ void write_bag(const dev_ctx& c, const embbag_args& a, int64_t g,
                                          const float (&acc)[VPL]) {
  const uint32_t d0 = lane() * VPL;
  const uint64_t slot = a.serve ? ((uint64_t)g & a.bag_mask) : (uint64_t)g;
  float* o = a.out + slot * a.dim + d0;
#pragma unroll
  for (int v = 0; v < VPL; ++v)
    if (d0 + v < a.dim) o[v] = acc[v];
  if (a.serve) {
    // the request is done when its last bag is written: push the outputs to host memory
    // first, then count the bag, then return the count to zero for the slot's next
    // request and raise the request's flag (system scope)
    // (the request's size is read before the bag is counted: once the count is complete
    // the host may hand the slot to a later request)
    fence_rel_sys();
    if (lane() == 0) {
      const uint64_t rs = a.bag_req[slot] & a.req_mask;
      const uint32_t nb = a.req_nbags[rs];
      const uint32_t k = add_rlx(a.req_cnt + rs, 1u) + 1;
      if (k == nb) {
        st_rlx(a.req_cnt + rs, 0u);
        fence_rel_sys();
        __hip_atomic_store(a.done + rs, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
      }
    }
  }
}

// Serving: waits until bag b is published (the device mirror holds the count).  Returns
// false when the session is stopped or aborted.  No device deadline: requests may arrive
// seconds apart; the host watchdog bounds the session.
__device__ __forceinline__ bool wait_published(const dev_ctx& c, const embbag_args& a, uint64_t b) {
  uint32_t n = 0;
  while (uni64(ld_rlx(a.pub_dev)) <= b) {
    if ((++n & 63) == 0) {
      if (aborted(c)) return false;
      if (uni(ld_rlx(a.pub_dev + 1))) return false;  // stop, mirrored from the host
    }
    __builtin_amdgcn_s_sleep(32);
  }
  fence_acq();
  return true;
}

// Next chunk after `d` (or the first one when !d.valid): continues the bag or grabs the
// next non-empty bag; empty bags get their zero output on the way.
// Takes the next bag into the held slot (or marks the source exhausted).
__device__ __forceinline__ void hold_next(const dev_ctx& c, const launch_t& li, const embbag_args& a,
                                          src_state& ss) {
  const int64_t A = ss.A, nb = ss.nb;
  const int64_t dealt = (int64_t)STATIC_ROUNDS * A < nb ? (int64_t)STATIC_ROUNDS * A : nb;
  int64_t g = -1;
  while (ss.dealt < STATIC_ROUNDS) {
    const int64_t s = (int64_t)ss.uw + (int64_t)ss.dealt * A;
    ++ss.dealt;
    if (s < dealt) {
      g = s;
      break;
    }
  }
  // never more partitions than waves: every partition then has a wave that starts in it
  // and stays until it is used up, so a bag is never left where no wave looks (a serving
  // wave that waits on an unpublished bag of its partition blocks only that partition)
  const uint32_t parts = (uint32_t)(A < (int64_t)WORK_PARTS ? A : (int64_t)WORK_PARTS);
  if (nb <= dealt) ss.tried = parts;  // every bag was dealt: no counter to visit
  while (g < 0 && ss.tried < parts) {
    const uint32_t p = (ss.uw + ss.tried) % parts;
    uint64_t v = 0;
    if (lane() == 0) v = add_rlx(counter(c, work_counter(p)), 1ull);
    v = rdlane64(v, 0);
    const int64_t b = dealt + (int64_t)v * parts + p;
    if (b < nb)
      g = b;
    else
      ++ss.tried;
  }
  if (g < 0) {
    ss.exhausted = true;
    ss.g = -1;
    return;
  }
  ss.g = g;
  const int64_t bag = a.list ? (int64_t)a.list[g] : g;
  ss.bag = bag;
  if (a.gather) {
    ss.j0 = bag * 64;
    ss.j1 = ((int64_t)a.n < ss.j0 + 64) ? (int64_t)a.n : ss.j0 + 64;
  } else if (!a.serve) {
    ss.j0 = a.off[bag];
    ss.j1 = a.off[bag + 1];
  }
  // a deferred bag: the resident-hit pass counted it in its launch total but did not
  // serve it
  if (a.list && lane() == 0) wcount(WS_DEFLEN, (uint64_t)(ss.j1 - ss.j0));
}

// Next chunk after `d` (or the first one when !d.valid): continues the bag or takes the
// held bag; empty bags get their zero output on the way.  With !may_wait, a held bag of
// an unpublished request ends the search (the wave first finishes what it has).
template <int VPL>
__device__ __forceinline__ desc_t next_desc(const dev_ctx& c, const launch_t& li, const embbag_args& a,
                            const desc_t& d, src_state& ss, bool may_wait) {
  desc_t r;
  r.valid = false;
  if (d.valid && !d.last) {
    r.g = d.g;
    r.j = d.j + d.n;
    r.end = d.end;
  } else {
    for (;;) {
      if (ss.g < 0) {
        if (ss.exhausted) return r;
        hold_next(c, li, a, ss);
        if (ss.g < 0) return r;
      }
      const int64_t g = ss.g, bag = ss.bag;
      int64_t j0 = ss.j0, j1 = ss.j1;
      if (a.serve) {
        // a claimed bag is read only once it is published (its ring slot may still hold
        // an older bag's entry until then)
        if (uni64(ld_rlx(a.pub_dev)) <= (uint64_t)bag) {
          if (!may_wait) return r;  // keep holding it
          if (!wait_published(c, a, (uint64_t)bag)) {
            ss.exhausted = true;
            ss.g = -1;
            return r;
          }
        } else {
          fence_acq();
        }
        const uint64_t slot = (uint64_t)bag & a.bag_mask;
        j0 = (int64_t)a.bag_j0[slot];
        j1 = (int64_t)a.bag_j1[slot];
      }
      // hold the next bag now, except near the end of the work: a held bag cannot go to
      // a wave that runs out, so the last bags are taken only when needed
      ss.g = -1;
      if (g + 2 * ss.A < ss.nb) hold_next(c, li, a, ss);
      if (j1 > j0) {
        r.g = bag;
        r.j = j0;
        r.end = j1;
        break;
      }
      if (!a.gather) {
        float z[VPL];
#pragma unroll
        for (int v = 0; v < VPL; ++v) z[v] = 0.0f;
        write_bag<VPL>(c, a, bag, z);
      }
    }
  }
  const int64_t left = r.end - r.j;
  r.n = (uint32_t)(left < 64 ? left : 64);
  r.last = r.j + r.n == r.end;
  r.valid = true;
  return r;
}

__device__ __forceinline__ void make_chunk(const dev_ctx& c, const embbag_args& a, const desc_t& d,
                                           chunk_t& ch) {
  ch.act = d.valid && lane() < d.n;
  ch.st = A_NONE;
  if (ch.act) {
    const uint64_t jl = (uint64_t)(d.j + lane());
    const int64_t row = a.idx[a.serve ? (jl & a.look_mask) : jl];
    uint64_t byte;
    if (a.gather) {
      byte = a.base_off + (uint64_t)row * a.row_bytes;
    } else {
      const uint32_t t = a.serve ? a.bag_tab[(uint64_t)d.g & a.bag_mask] : (uint32_t)(d.g % a.T);
      byte = a.base_off + (uint64_t)t * a.table_bytes + (uint64_t)row * a.row_bytes;
    }
    ch.line_id = (uint32_t)(byte >> c.line_shift);
    ch.off = (uint32_t)(byte & ((1ull << c.line_shift) - 1));
  }
}

// Row loads are device-coherent (they bypass any stale copy a previous tenant of the
// line left in this XCD's L2), so reads need no cache invalidation.
template <int VPL>
__device__ __forceinline__ void ld_row(const float* p, float (&v)[VPL]) {
  if constexpr (VPL == 1) {
    v[0] = __uint_as_float(ld_rlx(reinterpret_cast<const uint32_t*>(p)));
  } else {
#pragma unroll
    for (int h = 0; h < VPL / 2; ++h) {
      const uint64_t x = ld_rlx(reinterpret_cast<const uint64_t*>(p) + h);
      v[2 * h] = __uint_as_float((uint32_t)x);
      v[2 * h + 1] = __uint_as_float((uint32_t)(x >> 32));
    }
  }
}

// Rows per round of the consume loop (two rounds of row values are live at once).
template <int VPL>
constexpr uint32_t rows_per_round() { return VPL >= 4 ? 4u : 8u; }

// Loads rows [j, j + g) of the chunk (g <= R) into v; lanes past the row width read 0.
template <int VPL>
__device__ __forceinline__ void load_rows(const dev_ctx& c, const chunk_t& ch, uint32_t j, uint32_t g,
                                          uint32_t d0, bool mine, float (&v)[rows_per_round<VPL>()][VPL]) {
#pragma unroll
  for (uint32_t u = 0; u < rows_per_round<VPL>(); ++u) {
    if (u < g) {
      const uint32_t idx = rdlane(ch.idx, j + u);
      const uint32_t off = rdlane(ch.off, j + u);
      const float* p = reinterpret_cast<const float*>(line_ptr(c, idx) + off) + d0;
      if (mine) {
        ld_row<VPL>(p, v[u]);
      } else {
#pragma unroll
        for (int e = 0; e < VPL; ++e) v[u][e] = 0.0f;
      }
    }
  }
}

template <int VPL>
__device__ __forceinline__ void use_rows(const embbag_args& a, const desc_t& d, uint32_t j, uint32_t good,
                                         uint32_t d0, bool mine, const float (&v)[rows_per_round<VPL>()][VPL],
                                         float (&acc)[VPL]) {
#pragma unroll
  for (uint32_t u = 0; u < rows_per_round<VPL>(); ++u) {
    if (u < good && mine) {
      if (a.gather) {
        float* o = a.out + (uint64_t)(d.j + j + u) * a.dim + d0;
#pragma unroll
        for (int e = 0; e < VPL; ++e) o[e] = v[u][e];
      } else {
#pragma unroll
        for (int e = 0; e < VPL; ++e) acc[e] = acc[e] + fK(v[u][e], a.K);
      }
    }
  }
}

// Seqlock check of rows [j, j + g) of the chunk, issued only once the loads in `v` have
// returned: lane u re-reads the metadata of row j + u (unless the chunk pins it).  Returns
// the number of leading rows that are still valid.
template <int VPL>
__device__ __forceinline__ uint32_t validate_rows(const dev_ctx& c, const chunk_t& ch, uint32_t j, uint32_t g,
                                                  const float (&v)[rows_per_round<VPL>()][VPL]) {
  uint32_t dep = 0;
#pragma unroll
  for (uint32_t u = 0; u < rows_per_round<VPL>(); ++u)
    if (u < g) dep ^= __float_as_uint(v[u][0]);
  const uint32_t r = (j + lane()) & 63;
  uint32_t ridx = shfl32(ch.idx, r);
  const uint32_t rtag = shfl32(ch.line_id, r);
  const uint32_t rgen = shfl32(ch.gen, r);
  const uint32_t rpin = shfl32(ch.pinned ? 1u : 0u, r);
  // the metadata address depends on every row value of the round, so these loads are
  // issued after the row loads have completed (the seqlock order), and not before
  asm volatile("" : "+v"(ridx) : "v"(dep));
  bool bad = false;
  if (lane() < g && !rpin) bad = !line_still_valid(c, ridx, rtag, rgen);
  const uint64_t bm = ballot(bad);
  return bm ? ffs64(bm) : g;
}

// Consumes rows of the chunk in order until the first row whose lane has no line or
// (with `validate`) whose unpinned line changed tenant while it was read.  Returns the
// number of rows consumed.  Rows go in rounds; with validation the rounds are
// software-pipelined: the next round's row loads are in flight together with this
// round's metadata re-reads, so each round costs one memory round trip.
template <int VPL>
__device__ __forceinline__ uint32_t consume(const dev_ctx& c, const embbag_args& a, const desc_t& d,
                            const chunk_t& ch, float (&acc)[VPL], bool validate) {
  const uint64_t okm = ballot(ch.act && st_ok(ch.st));
  const uint32_t nok = (~okm == 0ull) ? 64u : ffs64(~okm);
  const uint32_t n = nok < d.n ? nok : d.n;
  const uint32_t d0 = lane() * VPL;
  const bool mine = d0 < a.dim;
  constexpr uint32_t R = rows_per_round<VPL>();
  if (!validate) {
    for (uint32_t j = 0; j < n; j += R) {
      const uint32_t g = (n - j) < R ? (n - j) : R;
      float v[R][VPL];
      load_rows<VPL>(c, ch, j, g, d0, mine, v);
      use_rows<VPL>(a, d, j, g, d0, mine, v, acc);
    }
    return n;
  }
  float va[R][VPL], vb[R][VPL];
  uint32_t j = 0;
  if (n) load_rows<VPL>(c, ch, 0, n < R ? n : R, d0, mine, va);
  while (j < n) {
    // round in va, next round into vb
    uint32_t g = (n - j) < R ? (n - j) : R;
    uint32_t jn = j + g;
    uint32_t gn = jn < n ? ((n - jn) < R ? (n - jn) : R) : 0;
    if (gn) load_rows<VPL>(c, ch, jn, gn, d0, mine, vb);
    uint32_t good = validate_rows<VPL>(c, ch, j, g, va);
    use_rows<VPL>(a, d, j, good, d0, mine, va, acc);
    if (good < g) return j + good;
    j = jn;
    if (j >= n) break;
    // round in vb, next round into va
    g = gn;
    jn = j + g;
    gn = jn < n ? ((n - jn) < R ? (n - jn) : R) : 0;
    if (gn) load_rows<VPL>(c, ch, jn, gn, d0, mine, va);
    good = validate_rows<VPL>(c, ch, j, g, vb);
    use_rows<VPL>(a, d, j, good, d0, mine, vb, acc);
    if (good < g) return j + good;
    j = jn;
  }
  return n;
}

// Consumes chunk `cc` of descriptor `dc` (already issued) into acc, in order, and writes
// the bag's output when dc is its last chunk.  A row whose unpinned line changed tenant
// while it was read (the seqlock check failed) is presented again optimistically, with
// the rest of the chunk, up to twice: waiting for the lines of a fresh claim is safe while
// this wave holds pins, since a claimed line always fills.  A row that met a full set, or
// keeps losing its line, is drained: the wave first drops every pin it holds (the other
// issued chunk `cn` included, if *n_issued; the caller then issues it again), then
// acquires the remaining rows one at a time while holding nothing, so that no wave ever
// waits for a line while it pins others (Sec. 2.3.2).  Returns false on abort/timeout.
template <int VPL>
__device__ __forceinline__ bool finish_chunk(const dev_ctx& c, const embbag_args& a, uint32_t q, desc_t dc,
                                             chunk_t& cc, float (&acc)[VPL], chunk_t& cn, bool& n_issued) {
  uint32_t k = 0;
  for (uint32_t attempt = 0;; ++attempt) {
    if (attempt) {
      dc.j += k;
      dc.n -= k;
      make_chunk(c, a, dc, cc);
      if (!chunk_issue(c, cc, q, true, PIN_NONE)) return false;
    }
    if (!chunk_wait(c, cc, false)) return false;
    const uint64_t t_cons = now();
    k = consume<VPL>(c, a, dc, cc, acc, true);
    chunk_release(c, cc, false);
    wtick(c, WS_T_CONSUME, t_cons);
    if (lane() == 0) wcount(WS_AUX1, k);
    if (k == dc.n || attempt == 2 || !st_ok(rdlane(cc.st, k))) break;
  }
  if (k < dc.n) {
    if (n_issued) {
      if (!chunk_wait(c, cn, false)) return false;
      chunk_release(c, cn, false);
      n_issued = false;
    }
    dc.j += k;
    dc.n -= k;
    while (dc.n > 0) {
      desc_t one = dc;
      one.n = 1;
      spin_t sp;
      for (;;) {
        make_chunk(c, a, one, cc);
        if (!chunk_issue(c, cc, q, true, PIN_LINE)) return false;
        if (rdlane(cc.st, 0) != A_EAGAIN) break;
        if (!sp.step(c, wi(W_WAY, (uint64_t)dc.g))) return false;
      }
      if (!chunk_wait(c, cc, false)) return false;
      consume<VPL>(c, a, one, cc, acc, false);
      chunk_release(c, cc, false);
      if (lane() == 0) wcount(WS_AUX1, 1);
      dc.j += 1;
      dc.n -= 1;
    }
  }
  if (dc.last && !a.gather) {
    write_bag<VPL>(c, a, dc.g, acc);
#pragma unroll
    for (int v = 0; v < VPL; ++v) acc[v] = 0.0f;
  }
  return true;
}

// One user wavefront of the embedding-bag / gather workload.  Both modes keep at most two
// chunks of reads in flight per wave, so they present the queues the same concurrency:
//  * asynchronous (Sec. 4.2): once the current chunk's lines are filled, the reads of the
//    next chunk are issued and then the current chunk is computed, so this wave's I/O
//    overlaps its own compute.  The next chunk is requested only after the current one
//    has arrived: the queues are first-come first-served at the store's IOPS cap, and a
//    prefetch queued earlier would stand in front of other waves' reads that are needed
//    now (it would not make the data arrive sooner, only later for someone else);
//  * synchronous (the plain method, array-like issue-and-wait): the reads of two chunks
//    are issued, both are waited for, then both are computed; the wave's compute never
//    overlaps its own I/O.
template <int VPL>
__device__ __forceinline__ void embbag_wave(const dev_ctx& c, const launch_t& li, const embbag_args& a, uint32_t uw,
                                            uint32_t active) {
  const uint32_t q = uw % c.num_qp;
  const bool async = a.mode == AGILE_MODE_ASYNC;
  float acc[VPL];
#pragma unroll
  for (int v = 0; v < VPL; ++v) acc[v] = 0.0f;
  desc_t none;
  none.valid = false;
  // a list launch runs the bags the resident-hit pass before it deferred
  const int64_t nb = a.list ? (int64_t)uni64(ld_rlx(counter(c, C_DEFER))) : (int64_t)a.nbags;
  src_state ss{-1, -1, 0, 0, false, uw, 0, 0, nb, (int64_t)active};
  chunk_t cc, cn;
  if (!async) {
    desc_t dc = next_desc<VPL>(c, li, a, none, ss, true);
    while (dc.valid) {
      make_chunk(c, a, dc, cc);
      if (!chunk_issue(c, cc, q, true, PIN_NONE)) return;
      // the pair's second chunk: the next one if it is already available
      desc_t dn = next_desc<VPL>(c, li, a, dc, ss, false);
      bool n_issued = false;
      if (dn.valid) {
        make_chunk(c, a, dn, cn);
        if (!chunk_issue(c, cn, q, true, PIN_NONE)) return;
        n_issued = true;
      }
      // every read of the pair completes before any of its compute
      if (!chunk_wait(c, cc, false)) return;
      if (n_issued && !chunk_wait(c, cn, false)) return;
      if (!finish_chunk<VPL>(c, a, q, dc, cc, acc, cn, n_issued)) return;
      if (dn.valid) {
        if (!n_issued) {  // dropped to drain the first chunk: issue it again
          make_chunk(c, a, dn, cn);
          if (!chunk_issue(c, cn, q, true, PIN_NONE)) return;
        }
        bool none_held = false;
        if (!finish_chunk<VPL>(c, a, q, dn, cn, acc, cc, none_held)) return;
        dc = dn;
      }
      const uint64_t t_desc = now();
      dc = next_desc<VPL>(c, li, a, dc, ss, true);
      wtick(c, WS_T_DESC, t_desc);
    }
    return;
  }
  desc_t dc = next_desc<VPL>(c, li, a, none, ss, true);
  if (!dc.valid) return;
  make_chunk(c, a, dc, cc);
  if (!chunk_issue(c, cc, q, true, PIN_NONE)) return;
  while (dc.valid) {
    if (!chunk_wait(c, cc, false)) return;
    desc_t dn;
    bool n_issued = false;
    const uint64_t t_desc = now();
    dn = next_desc<VPL>(c, li, a, dc, ss, false);
    if (dn.valid) {
      make_chunk(c, a, dn, cn);
      wtick(c, WS_T_DESC, t_desc);
      if (!chunk_issue(c, cn, q, true, PIN_NONE)) return;
      n_issued = true;
    } else {
      wtick(c, WS_T_DESC, t_desc);
    }
    if (!finish_chunk<VPL>(c, a, q, dc, cc, acc, cn, n_issued)) return;
    const uint64_t t_next = now();
    if (!dn.valid && ss.g >= 0) dn = next_desc<VPL>(c, li, a, dc, ss, true);
    dc = dn;
    if (!dc.valid) break;
    if (n_issued) {
      cc = cn;
      wtick(c, WS_T_DESC, t_next);
    } else {
      make_chunk(c, a, dc, cc);
      wtick(c, WS_T_DESC, t_next);
      if (!chunk_issue(c, cc, q, true, PIN_NONE)) return;
    }
  }
}

// Serialized mode: lane 0 of a single wave handles one lookup at a time in program order
// (issue, wait, compute, release), so the cache sees exactly the request sequence.
template <int VPL>
__device__ __forceinline__ void embbag_serial(const dev_ctx& c, const launch_t& li, const embbag_args& a) {
  float acc[VPL];
  const uint64_t nb = a.nbags;
  for (uint64_t g = 0; g < nb; ++g) {
    int64_t j0 = a.gather ? (int64_t)g * 64 : a.off[g];
    int64_t j1 = a.gather ? (((int64_t)a.n < j0 + 64) ? (int64_t)a.n : j0 + 64) : a.off[g + 1];
#pragma unroll
    for (int v = 0; v < VPL; ++v) acc[v] = 0.0f;
    for (int64_t j = j0; j < j1; ++j) {
      desc_t d;
      d.g = (int64_t)g;
      d.j = j;
      d.end = j + 1;
      d.n = 1;
      d.valid = true;
      d.last = true;
      chunk_t ch;
      spin_t sp;
      for (;;) {
        make_chunk(c, a, d, ch);
        if (!chunk_issue(c, ch, 0, true, PIN_LINE)) return;
        if (!chunk_wait(c, ch, false)) return;
        const uint32_t k = consume<VPL>(c, a, d, ch, acc, false);
        chunk_release(c, ch, false);
        if (k == 1) {
          if (lane() == 0) wcount(WS_AUX1, 1);
          break;
        }
        if (!sp.step(c, wi(W_WAY, 0))) return;
      }
    }
    if (!a.gather) write_bag<VPL>(c, a, (int64_t)g, acc);
  }
}

// ---- resident-hit pass: the first of the two launches of every embedding-bag / gather call
// A lean loop with no pins, no locks and no queue traffic: each wave takes whole bags
// and, chunk by chunk, probes the sets of the chunk's lines (the LDS-staged probe), and
// if every line is resident with its data (READY, MODIFIED or being written back) reads
// the rows optimistically, adds them in order and checks the lines' tags and generations
// once the loads have completed (the seqlock order).  A bag with a line that is absent
// or still being fetched, or whose line changed tenant while it was read, is appended to
// the deferred list and left entirely to the I/O launch that follows on the stream (which
// recomputes it from the start, so the two launches never split a bag's sum).  Hits here
// count as requests and hits like any other.
// Rows [r, r + g) of a chunk whose lane u holds the address of row u: the row's address
// is made uniform with two lane reads, and every lane loads its own columns of it.
template <int VPL>
__device__ __forceinline__ void hit_load(uint64_t raddr, uint32_t r, uint32_t g, uint32_t d0, bool mine,
                                         float (&v)[rows_per_round<VPL>()][VPL]) {
#pragma unroll
  for (uint32_t u = 0; u < rows_per_round<VPL>(); ++u) {
    if (u < g) {
      const uint64_t p = ((uint64_t)rdlane((uint32_t)(raddr >> 32), r + u) << 32) |
                         rdlane((uint32_t)raddr, r + u);
      if (mine) {
        ld_row<VPL>(reinterpret_cast<const float*>(p) + d0, v[u]);
      } else {
#pragma unroll
        for (int e = 0; e < VPL; ++e) v[u][e] = 0.0f;
      }
    }
  }
}
// Adds (or, gathering, writes out) rows [r, r + g) held in v; lookup j of the chunk's
// first row gives the gather output position.
template <int VPL>
__device__ __forceinline__ void hit_use(const embbag_args& a, int64_t j, uint32_t g, uint32_t d0, bool mine,
                                        const float (&v)[rows_per_round<VPL>()][VPL], float (&acc)[VPL]) {
  if (!mine) return;
  if (a.gather) {
#pragma unroll
    for (uint32_t u = 0; u < rows_per_round<VPL>(); ++u)
      if (u < g) {
        float* o = a.out + (uint64_t)(j + u) * a.dim + d0;
#pragma unroll
        for (int e = 0; e < VPL; ++e) o[e] = v[u][e];
      }
  } else if (a.K == 0) {
#pragma unroll
    for (uint32_t u = 0; u < rows_per_round<VPL>(); ++u)
      if (u < g) {
#pragma unroll
        for (int e = 0; e < VPL; ++e) acc[e] = acc[e] + v[u][e];
      }
  } else {
#pragma unroll
    for (uint32_t u = 0; u < rows_per_round<VPL>(); ++u)
      if (u < g) {
#pragma unroll
        for (int e = 0; e < VPL; ++e) acc[e] = acc[e] + fK(v[u][e], a.K);
      }
  }
}

// One wavefront per bag and per workgroup, so the hardware's dispatch of workgroups
// balances bags of uneven length, no wave waits on a work counter, and a short bag's
// slot is free as soon as the bag is done (with 4 or 2 bags to a workgroup the slot
// waits for the workgroup's longest bag: the DLRM-style hit replay took 0.100 or
// 0.090 ms against 0.087 ms, and 2.74 or 2.19 ms against 1.91 ms at K = 256).  Each wave
// has its own 8 KiB LDS area for the staged probe.  Four wavefronts per SIMD (up to 128
// registers): at five the loop spills, and the spills cost more than the fifth wave
// gains (0.144 ms against 0.100 ms, 4 bags to a workgroup).
constexpr uint32_t HIT_WAVES = 1;
struct alignas(16) hit_lds_t {
  uint8_t b[HIT_WAVES][PROBE_LDS];
};
// From this K on, each round of rows is checked right after it has loaded and before it
// is computed, so that a line evicted during a long computation costs nothing (the rows
// already read stay valid); below it one check per chunk, after every row has been used,
// keeps the loads of consecutive rounds in flight together.
constexpr uint32_t EARLY_CHECK_K = 256;

// Serves lookups [j0, j1) of bag g from resident lines into acc, chunk by chunk, and
// writes the bag's output when it gets to the end.  Returns the first lookup it did not
// consume: a chunk with a line that is absent or still being fetched stops it at the
// chunk's start, a row whose line changed tenant while it was read at that row's round
// (K >= EARLY_CHECK_K) or at the chunk's start (smaller K); acc then holds exactly the
// lookups before that position.
template <int VPL>
__device__ __forceinline__ int64_t hit_bag_part(const dev_ctx& c, const embbag_args& a, uint64_t g, uint8_t* lds,
                                                float (&acc)[VPL], int64_t j0, int64_t j1) {
  const uint32_t d0 = lane() * VPL;
  const bool mine = d0 < a.dim;
  constexpr uint32_t R = rows_per_round<VPL>();
  const uint64_t lmask = (1ull << c.line_shift) - 1;
  const uint32_t t = a.gather ? 0u : (uint32_t)(g % a.T);
  const bool early = a.K >= EARLY_CHECK_K;
  for (int64_t j = j0; j < j1; j += 64) {
    const uint32_t n = (uint32_t)((j1 - j) < 64 ? (j1 - j) : 64);
    chunk_t ch;
    ch.act = lane() < n;
    ch.pinned = false;
    ch.line_id = 0;
    ch.off = 0;
    if (ch.act) {
      const int64_t row = a.idx[j + lane()];
      const uint64_t byte = a.base_off + (uint64_t)t * a.table_bytes + (uint64_t)row * a.row_bytes;
      ch.line_id = (uint32_t)(byte >> c.line_shift);
      ch.off = (uint32_t)(byte & lmask);
    }
    const uint32_t base = ch.act ? set_of(c, ch.line_id) * c.assoc : 0u;
    uint64_t m = 0;
    int w = -1;
    if (probe_staged_ok(c.assoc))
      w = probe_staged(c, ch.act, base, ch.line_id, m, lds);
    else if (ch.act)
      w = probe_set(c, base, ch.line_id, m);
    const bool hit = ch.act && w >= 0 && m_valid_data(m_state(m));
    if (ballot(ch.act && !hit)) return j;
    ch.idx = base + (uint32_t)(w < 0 ? 0 : w);
    ch.gen = m_gen(m);
    if (ch.act && !(m & M_REF)) or_rlx(c.meta + ch.idx, M_REF);
    // each lane's row address, so a row costs two lane reads and one load
    const uint64_t raddr = (uint64_t)(uintptr_t)line_ptr(c, ch.idx) + ch.off;
    float va[R][VPL], vb[R][VPL];
    if (early) {
      for (uint32_t r = 0; r < n; r += R) {
        const uint32_t gr = (n - r) < R ? (n - r) : R;
        hit_load<VPL>(raddr, r, gr, d0, mine, va);
        // the round's loads have completed before its lines are looked at again
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
        asm volatile("" ::: "memory");
        const uint32_t src = (r + lane()) & 63;
        const uint32_t vidx = shfl32(ch.idx, src), vtag = shfl32(ch.line_id, src), vgen = shfl32(ch.gen, src);
        if (ballot(lane() < gr && !line_still_valid(c, vidx, vtag, vgen))) return j + r;
        hit_use<VPL>(a, j + r, gr, d0, mine, va, acc);
      }
      continue;
    }
    float acc0[VPL];
#pragma unroll
    for (int v = 0; v < VPL; ++v) acc0[v] = acc[v];
    // the rows in rounds of R, two rounds in flight, added as they arrive
    hit_load<VPL>(raddr, 0, n < R ? n : R, d0, mine, va);
    for (uint32_t r = 0; r < n;) {
      uint32_t gcur = (n - r) < R ? (n - r) : R;
      uint32_t rn = r + gcur;
      uint32_t gn = rn < n ? ((n - rn) < R ? (n - rn) : R) : 0;
      if (gn) hit_load<VPL>(raddr, rn, gn, d0, mine, vb);
      hit_use<VPL>(a, j + r, gcur, d0, mine, va, acc);
      r = rn;
      if (r >= n) break;
      gcur = gn;
      rn = r + gcur;
      gn = rn < n ? ((n - rn) < R ? (n - rn) : R) : 0;
      if (gn) hit_load<VPL>(raddr, rn, gn, d0, mine, va);
      hit_use<VPL>(a, j + r, gcur, d0, mine, vb, acc);
      r = rn;
    }
    // every row load of this wave has completed before the metadata is read again
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    asm volatile("" ::: "memory");
    const bool bad = ch.act && !line_still_valid(c, ch.idx, ch.line_id, ch.gen);
    if (ballot(bad)) {
#pragma unroll
      for (int v = 0; v < VPL; ++v) acc[v] = acc0[v];
      return j;
    }
  }
  if (!a.gather) write_bag<VPL>(c, a, (int64_t)g, acc);
  return j1;
}

// The whole bag g from resident lines, or false (nothing written).
template <int VPL>
__device__ __forceinline__ bool hit_bag(const dev_ctx& c, const embbag_args& a, uint64_t g, uint8_t* lds) {
  int64_t j0, j1;
  if (a.gather) {
    j0 = (int64_t)g * 64;
    j1 = ((int64_t)a.n < j0 + 64) ? (int64_t)a.n : j0 + 64;
  } else {
    j0 = a.off[g];
    j1 = a.off[g + 1];
  }
  float acc[VPL];
#pragma unroll
  for (int v = 0; v < VPL; ++v) acc[v] = 0.0f;
  return hit_bag_part<VPL>(c, a, g, lds, acc, j0, j1) == j1;
}

// The resident-hit pass: bag g = workgroup * HIT_WAVES + wave.  It carries no service
// wavefronts and none of the I/O path's code; a bag it cannot serve goes to the
// deferred list.
template <int VPL>
__global__ __launch_bounds__(64 * HIT_WAVES, 4) void k_embbag_hit(dev_ctx c, embbag_args a, uint32_t* list) {
  __shared__ hit_lds_t lds;
  const uint64_t g = (uint64_t)blockIdx.x * HIT_WAVES + threadIdx.x / 64;
  if (g >= a.nbags) return;
  if (!hit_bag<VPL>(c, a, g, lds.b[threadIdx.x / 64]) && lane() == 0)
    list[add_rlx(counter(c, C_DEFER), 1ull)] = (uint32_t)g;
}

// ---- next-batch prefetch (Sec. 4.3's asynchronous DLRM mode: the data of the next epoch
// is requested while the current one computes)
// One launch carries the service wavefronts, a few prefetch wavefronts and the compute
// loop over the current batch.  The prefetch wavefronts walk the next batch's lookups 64
// at a time and claim the lines that are neither resident nor in flight without pinning
// them (a full set drops the request): they never wait for data, only for queue slots
// and for the store's backlog to fall below its bound, so the store is kept busy by them
// while every other wavefront computes.  Once their share is submitted they join the
// compute loop (in a launch of few wavefronts every wave prefetches and computes in
// turns; the backward's launch carries the same prefetch role).  The compute loop takes whole bags
// from work counters and serves each from resident lines as the resident-hit pass does
// (optimistic reads, checked after loading); where that stops (a line absent or in
// flight, or a line that changed tenant), the same wavefront goes on with the rest of
// the bag through the cache and the queues (issue, wait, consume, as the I/O launch
// does), so no bag waits for a second launch.
struct pf_args {
  const int64_t* idx;  // the next batch's lookups
  const int64_t* off;  // its bag offsets [nbags + 1]
  uint64_t nbags;      // its bags; 0: nothing to prefetch
  uint64_t store_bytes;
  uint64_t base_off, table_bytes;  // the tables (bag g is of table g mod T)
  uint32_t row_bytes, T;
  uint64_t backlog;    // commands in flight (all queues) above which prefetching pauses
  uint32_t waves;      // user wavefronts that prefetch
  uint32_t interleave; // they prefetch and compute in turns (else prefetch, then compute)
};

// The bag holding lookup j: the g with off[g] <= j < off[g + 1] (off[0] <= j < off[nb]).
__device__ __forceinline__ uint64_t bag_of(const int64_t* off, uint64_t nb, int64_t j) {
  uint64_t lo = 0, hi = nb;
  while (hi - lo > 1) {
    const uint64_t mid = (lo + hi) >> 1;
    if (off[mid] <= j)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// The bag of each lane's lookup j = j0 + lane (all lanes take part; j0 < off[nb]): the
// bag of j0 by a 64-ary search over the offsets (one wave-wide round per factor of 64),
// then a lane's own bag from the next 64 offsets, held one per lane, by a 6-step search
// among them (the number of bag boundaries in (j0, j]).  A lane whose lookup lies past
// those 64 boundaries (a run of empty bags) searches the offsets alone.
__device__ __forceinline__ uint64_t chunk_bags(const int64_t* off, uint64_t nb, int64_t j0, int64_t j) {
  uint64_t lo = 0, hi = nb;  // off[lo] <= j0 < off[hi]
  while (hi - lo > 1) {
    const uint64_t step = (hi - lo + 63) / 64;
    const uint64_t p = lo + (uint64_t)lane() * step;
    const uint64_t m = ballot(p < hi && off[p] <= j0);
    const uint64_t nlo = lo + (uint64_t)(63 - __builtin_clzll(m)) * step;
    hi = (nlo + step < hi) ? nlo + step : hi;
    lo = nlo;
  }
  const uint64_t bi = lo + 1 + lane();
  const uint64_t bnd = bi <= nb ? (uint64_t)off[bi] : ~0ull;  // offsets are >= 0
  uint32_t cnt = 0;
#pragma unroll
  for (uint32_t st = 32; st; st >>= 1)
    if (shfl64(bnd, cnt + st - 1) <= (uint64_t)j) cnt += st;
  if (cnt == 63 && shfl64(bnd, 63) <= (uint64_t)j) return j < off[nb] ? bag_of(off, nb, j) : nb;
  return lo + cnt;
}

// The store's backlog (commands submitted and not yet completed, all queues) is at the
// prefetch's bound.  The store serves its queues first come, first served: a bounded
// backlog keeps it busy while the reads that computing waves need now wait behind
// little of it.
__device__ __forceinline__ bool backlog_full(const dev_ctx& c, const pf_args& p) {
  return uni64(ld_rlx(counter(c, C_SUBMITTED))) - uni64(ld_rlx(counter(c, C_COMPLETED))) >= p.backlog;
}

// Claims (unpinned) the lines of the next batch's lookups [j0, j0 + 64) that are neither
// resident nor in flight, and submits their READs.  False on abort or time-out.
__device__ __forceinline__ bool prefetch_chunk(const dev_ctx& c, const pf_args& p, uint32_t q, int64_t j0,
                                               int64_t j_hi) {
  const uint64_t lmask = (1ull << c.line_shift) - 1;
  chunk_t ch;
  const int64_t j = j0 + lane();
  ch.act = j < j_hi;
  ch.pinned = false;
  ch.line_id = 0;
  ch.off = 0;
  const uint64_t g = chunk_bags(p.off, p.nbags, j0, j);
  if (ch.act) {
    const uint64_t byte = p.base_off + (g % p.T) * p.table_bytes + (uint64_t)p.idx[j] * p.row_bytes;
    ch.act = byte < p.store_bytes;  // a hint: a row outside the store is not fetched
    ch.line_id = (uint32_t)(byte >> c.line_shift);
    ch.off = (uint32_t)(byte & lmask);
  }
  return chunk_issue(c, ch, q, false, PIN_PREFETCH);
}

// A dedicated prefetch wave's share: chunks w, w + P, ... of the next batch (P = p.waves),
// each after the backlog is below its bound.
__device__ __forceinline__ bool prefetch_wave(const dev_ctx& c, const pf_args& p, uint32_t w) {
  const int64_t j_lo = p.off[0], j_hi = p.off[p.nbags];
  const uint32_t q = w % c.num_qp;
  for (int64_t j0 = j_lo + (int64_t)w * 64; j0 < j_hi; j0 += (int64_t)p.waves * 64) {
    spin_t sp;
    while (backlog_full(c, p))
      if (!sp.step(c, wi(W_BACKLOG, p.backlog))) return false;
    if (!prefetch_chunk(c, p, q, j0, j_hi)) return false;
  }
  return true;
}

// Lookups [j, j1) of bag g through the cache and the queues, one chunk at a time, added
// to acc; writes the bag's output.  False on abort or time-out.
template <int VPL>
__device__ __forceinline__ bool io_rest(const dev_ctx& c, const embbag_args& a, uint32_t q, int64_t g, int64_t j,
                                        int64_t j1, float (&acc)[VPL]) {
  chunk_t cc, cn;
  while (j < j1) {
    desc_t d;
    d.g = g;
    d.j = j;
    d.end = j1;
    d.n = (uint32_t)((j1 - j) < 64 ? (j1 - j) : 64);
    d.last = j + d.n == j1;
    d.valid = true;
    make_chunk(c, a, d, cc);
    if (!chunk_issue(c, cc, q, true, PIN_NONE)) return false;
    bool none_held = false;
    if (!finish_chunk<VPL>(c, a, q, d, cc, acc, cn, none_held)) return false;
    j += d.n;
  }
  return true;
}

// The compute loop over work counters: wave uw of nw starts in partition uw mod P
// (P = min(WORK_PARTS, nw); bag g belongs to partition g mod P) and moves on when it is
// used up.  The lookups that go through the queues are counted as such (and taken out
// of the resident-hit total the launch adds).  compute_bag takes and computes the
// wave's next bag: 1 done, 0 no bag left, -1 abort or time-out.
template <int VPL>
__device__ __forceinline__ int compute_bag(const dev_ctx& c, const embbag_args& a, uint32_t uw, uint32_t nw,
                                           uint32_t& t) {
  const uint32_t parts = nw < WORK_PARTS ? nw : WORK_PARTS;
  while (t < parts) {
    const uint32_t pp = (uw + t) % parts;
    uint64_t v = 0;
    if (lane() == 0) v = add_rlx(counter(c, work_counter(pp)), 1ull);
    const uint64_t g = rdlane64(v, 0) * parts + pp;
    if (g >= a.nbags) {
      ++t;
      continue;
    }
    const int64_t j0 = a.off[g], j1 = a.off[g + 1];
    float acc[VPL];
#pragma unroll
    for (int e = 0; e < VPL; ++e) acc[e] = 0.0f;
    const int64_t j = hit_bag_part<VPL>(c, a, g, probe_area(), acc, j0, j1);
    if (j < j1) {
      if (lane() == 0) wcount(WS_DEFLEN, (uint64_t)(j1 - j));
      if (!io_rest<VPL>(c, a, uw % c.num_qp, (int64_t)g, j, j1, acc)) return -1;
    }
    return 1;
  }
  return 0;
}

// With few wavefronts in the launch every wave prefetches and computes, in turns: it
// tops the store's backlog up with its next chunks of the next batch, computes one bag,
// and so on; once its bags are gone it finishes its chunks.  (With many wavefronts a few
// dedicated prefetch waves keep the store busy and the others never stop computing.)
template <int VPL>
__device__ __forceinline__ void pf_interleaved(const dev_ctx& c, const embbag_args& a, const pf_args& p, uint32_t uw,
                                               uint32_t nw) {
  const int64_t j_hi = p.off[p.nbags];
  const uint32_t q = uw % c.num_qp;
  int64_t pj = p.off[0] + (int64_t)uw * 64;
  uint32_t t = 0;
  bool comp = a.nbags > 0;
  while (pj < j_hi || comp) {
    while (pj < j_hi && !backlog_full(c, p)) {
      if (!prefetch_chunk(c, p, q, pj, j_hi)) return;
      pj += (int64_t)p.waves * 64;
    }
    if (comp) {
      const int r = compute_bag<VPL>(c, a, uw, nw, t);
      if (r < 0) return;
      comp = r > 0;
      continue;
    }
    spin_t sp;
    while (pj < j_hi && backlog_full(c, p))
      if (!sp.step(c, wi(W_BACKLOG, p.backlog))) return;
  }
}

template <int VPL>
__global__ __launch_bounds__(WG) void k_embbag_pf(dev_ctx c, launch_t li, embbag_args a, pf_args p) {
  if (blockIdx.x < li.service_blocks) {
    run_service(c, li);
    return;
  }
  user_wave_begin();
  const uint32_t uw = (blockIdx.x - li.service_blocks) * WPB + threadIdx.x / 64;
  if (uw == 0 && lane() == 0 && a.nbags)
    add_rlx(counter(c, C_HIT_TOTAL), (uint64_t)(a.off[a.nbags] - a.off[0]));
  if (uw < a.active_waves) {
    const bool pfw = uw < p.waves && p.nbags;
    if (pfw && p.interleave) {
      pf_interleaved<VPL>(c, a, p, uw, a.active_waves);
    } else {
      bool ok = true;
      if (pfw) ok = prefetch_wave(c, p, uw);
      uint32_t t = 0;
      if (ok && a.nbags)
        while (compute_bag<VPL>(c, a, uw, a.active_waves, t) > 0) {
        }
    }
  }
  user_wave_done(c, li);
}

// Embedding-bag forward over a copy of the tables resident in device memory: no cache,
// queues or service wavefronts (the kernel-only side of a Sec. 4.5-style breakdown, and
// the ceiling the cached hit path is measured against).  One wavefront per bag, four per
// workgroup, so the hardware's dispatch of workgroups balances bags of uneven length.
// Lane l holds elements [l*VPL, l*VPL + VPL) of the row; a bag's indices are loaded 64
// at a time (one per lane) and its rows R at a time, all R loads in flight together.
// The same arithmetic, in the same order, as the cached path: out = sum over the bag's
// lookups, in order, of f_K(row), from +0.0f.
constexpr uint32_t RES_WAVES = 4;
template <int VPL>
__global__ __launch_bounds__(64 * RES_WAVES) void k_embbag_resident(dev_ctx c, const uint8_t* img, embbag_args a) {
  constexpr uint32_t R = 8;
  const uint64_t bag = (uint64_t)blockIdx.x * RES_WAVES + threadIdx.x / 64;
  if (bag >= a.nbags) return;
  const int64_t j0 = a.off[bag], j1 = a.off[bag + 1];
  const uint8_t* tab = img + a.base_off + (uint64_t)(bag % a.T) * a.table_bytes;
  const uint32_t d0 = lane() * VPL;
  const bool mine = d0 < a.dim;
  float acc[VPL];
#pragma unroll
  for (int e = 0; e < VPL; ++e) acc[e] = 0.0f;
  for (int64_t j = j0; j < j1; j += 64) {
    const uint32_t n = (uint32_t)(j1 - j < 64 ? j1 - j : 64);
    int64_t row = 0;
    if (lane() < n) {
      row = a.idx[j + lane()];
      if ((uint64_t)row >= a.rows) {
        raise_error(c, E_STATE, (uint64_t)row);
        row = -1;  // contributes nothing
      }
    }
    for (uint32_t u = 0; u < n; u += R) {
      float v[R][VPL];
#pragma unroll
      for (uint32_t k = 0; k < R; ++k) {
        const int64_t r = (int64_t)rdlane64((uint64_t)row, u + k < n ? u + k : 0);
        const bool ok = u + k < n && r >= 0 && mine;
        const float* p = reinterpret_cast<const float*>(tab + (uint64_t)(ok ? r : 0) * a.row_bytes) + d0;
        if constexpr (VPL == 1) {
          v[k][0] = ok ? p[0] : 0.0f;
        } else {
#pragma unroll
          for (int h = 0; h < VPL / 2; ++h) {
            float2 w = make_float2(0.0f, 0.0f);
            if (ok) w = reinterpret_cast<const float2*>(p)[h];
            v[k][2 * h] = w.x;
            v[k][2 * h + 1] = w.y;
          }
        }
      }
#pragma unroll
      for (uint32_t k = 0; k < R; ++k) {
        const int64_t r = (int64_t)rdlane64((uint64_t)row, u + k < n ? u + k : 0);
        if (u + k < n && r >= 0) {
#pragma unroll
          for (int e = 0; e < VPL; ++e) acc[e] += fK(v[k][e], a.K);
        }
      }
    }
  }
  float* o = a.out + bag * a.dim + d0;
#pragma unroll
  for (int e = 0; e < VPL; ++e)
    if (d0 + e < a.dim) o[e] = acc[e];
}

// A launch that runs the deferred list of the resident-hit pass before it sizes itself by
// the list (its count is final when the launch starts): only the leading user
// workgroups that give one wave per deferred bag take part (at least one workgroup), the
// others leave at once, and the service waits for the ones taking part.  A replay whose
// bags were all served costs one workgroup and the service instead of the whole grid.
template <int VPL>
__global__ __launch_bounds__(WG) void k_embbag(dev_ctx c, launch_t li, embbag_args a) {
  uint32_t active = a.active_waves;
  if (a.list) {
    const uint64_t nd = uni64(ld_rlx(counter(c, C_DEFER)));
    const uint64_t need = ((nd > WPB ? nd : WPB) + WPB - 1) / WPB * WPB;
    if (need < li.user_waves) li.user_waves = (uint32_t)need;
    if (li.user_waves < active) active = li.user_waves;
  }
  if (blockIdx.x < li.service_blocks) {
    run_service(c, li);
    return;
  }
  if ((blockIdx.x - li.service_blocks) * WPB >= li.user_waves) return;  // the whole workgroup
  user_wave_begin();
  const uint32_t uw = (blockIdx.x - li.service_blocks) * WPB + threadIdx.x / 64;
  if (a.list && uw == 0 && lane() == 0)
    add_rlx(counter(c, C_HIT_TOTAL), a.gather ? a.n : (uint64_t)(a.off[a.nbags] - a.off[0]));
  if (c.flags & AGILE_F_SERIALIZED) {
    if (uw == 0) embbag_serial<VPL>(c, li, a);
  } else if (uw < active) {
    embbag_wave<VPL>(c, li, a, uw, active);
  }
  user_wave_done(c, li);
}

// Serving kernel: the embedding-bag wave loop over a stream of requests.  One extra
// service wavefront stages what the host publishes: it takes the host's count of bags
// with acquire (system scope), copies the new bags' descriptors, their lookups and their
// requests' sizes from the rings in pinned host memory into the same slots of HBM rings,
// and passes the count on with release, so the waves read HBM, not PCIe.  It also
// mirrors the stop flag and the host's abort flag.
struct serve_stage {
  const uint64_t *h_j0, *h_j1, *h_req;  // the host's rings (pinned, mapped)
  const uint32_t *h_tab, *h_rnb;
  const int64_t* h_idx;
  uint64_t *d_j0, *d_j1, *d_req;        // their HBM copies, read by the waves
  uint32_t *d_tab, *d_rnb;
  int64_t* d_idx;
  uint64_t* pub_dev;                    // [0] bags staged, [1] stop
};
__device__ __forceinline__ void stage_published(const dev_ctx& c, const embbag_args& a, const serve_stage& st) {
  uint64_t last = 0;
  for (;;) {
    const uint64_t v = uni64(__hip_atomic_load(a.pub_host, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM));
    if (v != last) {
      for (uint64_t b = last + lane(); b < v; b += 64) {
        const uint64_t sl = b & a.bag_mask;
        st.d_j0[sl] = ring_ld(st.h_j0 + sl);
        st.d_j1[sl] = ring_ld(st.h_j1 + sl);
        st.d_req[sl] = ring_ld(st.h_req + sl);
        st.d_tab[sl] = ring_ld(st.h_tab + sl);
      }
      // the new bags' lookups are one run of positions, their requests one run of
      // numbers (the host publishes whole requests)
      const uint64_t jl = uni64(ring_ld(st.h_j0 + (last & a.bag_mask)));
      const uint64_t jh = uni64(ring_ld(st.h_j1 + ((v - 1) & a.bag_mask)));
      for (uint64_t j0 = jl; j0 < jh; j0 += 8 * 64) {
        int64_t x[8];
#pragma unroll
        for (uint32_t k = 0; k < 8; ++k) {
          const uint64_t j = j0 + k * 64 + lane();
          if (j < jh) x[k] = ring_ld(st.h_idx + (j & a.look_mask));
        }
#pragma unroll
        for (uint32_t k = 0; k < 8; ++k) {
          const uint64_t j = j0 + k * 64 + lane();
          if (j < jh) st.d_idx[j & a.look_mask] = x[k];
        }
      }
      const uint64_t rl = uni64(ring_ld(st.h_req + (last & a.bag_mask)));
      const uint64_t rh = uni64(ring_ld(st.h_req + ((v - 1) & a.bag_mask)));
      for (uint64_t r = rl + lane(); r <= rh; r += 64) st.d_rnb[r & a.req_mask] = ring_ld(st.h_rnb + (r & a.req_mask));
      last = v;
      fence_rel();  // the copies before the count that publishes them
      if (lane() == 0) __hip_atomic_store(st.pub_dev, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (aborted(c) || host_abort_poll(c)) break;
    if (uni64(__hip_atomic_load(a.pub_host + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM))) {
      if (lane() == 0) st_rlx(st.pub_dev + 1, 1ull);
      break;
    }
    __builtin_amdgcn_s_sleep(16);
  }
}

template <int VPL>
__global__ __launch_bounds__(WG) void k_serve(dev_ctx c, launch_t li, embbag_args a, serve_stage st) {
  if (blockIdx.x < li.service_blocks) {
    if (service_role(li) == li.n_ctrl + li.n_cq) {
      stage_published(c, a, st);
      return;
    }
    run_service(c, li);
    return;
  }
  user_wave_begin();
  const uint32_t uw = (blockIdx.x - li.service_blocks) * WPB + threadIdx.x / 64;
  if (uw < a.active_waves) embbag_wave<VPL>(c, li, a, uw, a.active_waves);
  user_wave_done(c, li);
}

// ---- host-level ticket API kernels
__global__ __launch_bounds__(WG) void k_async_read(dev_ctx c, launch_t li, const uint64_t* blocks,
                                                   uint32_t n, agile_ticket* tickets) {
  if (blockIdx.x < li.service_blocks) {
    run_service(c, li);
    return;
  }
  user_wave_begin();
  const uint32_t uw = (blockIdx.x - li.service_blocks) * WPB + threadIdx.x / 64;
  const uint32_t q = uw % c.num_qp;
  for (uint64_t base = (uint64_t)uw * 64; base < n; base += (uint64_t)li.user_waves * 64) {
    chunk_t ch;
    const uint64_t i = base + lane();
    ch.act = i < n;
    uint64_t blk = 0;
    if (ch.act) {
      blk = blocks[i];
      if (blk >= c.store_blocks) {
        raise_error(c, E_STATE, blk);
        ch.act = false;
      }
      ch.line_id = (uint32_t)(blk / c.blocks_per_line);
      ch.off = (uint32_t)((blk % c.blocks_per_line) << 12);
    }
    if (!chunk_issue(c, ch, q, true, PIN_EACH)) break;
    if (ch.act) {
      const bool ok = ch.st == A_HIT || ch.st == A_JOIN || ch.st == A_MISS;
      tickets[i] = (uint64_t)ch.idx | ((uint64_t)(ch.gen & 0xFF) << 32) |
                   ((uint64_t)(ok ? TK_OK : TK_EAGAIN) << 40) | ((uint64_t)(ch.off >> 12) << 48);
    }
  }
  user_wave_done(c, li);
}

__global__ __launch_bounds__(WG) void k_wait(dev_ctx c, launch_t li, const agile_ticket* tickets,
                                             uint32_t n, void** ptrs) {
  user_wave_begin();
  const uint32_t uw = blockIdx.x * WPB + threadIdx.x / 64;
  const uint64_t i = (uint64_t)uw * 64 + lane();
  bool waiting = false;
  uint32_t idx = 0, gen = 0, st = TK_EAGAIN, boff = 0;
  if (i < n) {
    const uint64_t t = tickets[i];
    idx = (uint32_t)t;
    gen = (uint32_t)(t >> 32) & 0xFF;
    st = (uint32_t)(t >> 40) & 0xFF;
    boff = (uint32_t)(t >> 48);
    if (st == TK_OK) {
      if (idx >= c.num_lines) {
        raise_error(c, E_STATE, t);
      } else {
        waiting = true;
      }
    }
  }
  spin_t sp;
  bool okay = true;
  while (ballot(waiting)) {
    if (waiting) {
      const uint64_t m = ld_rlx(c.meta + idx);
      if (m_state(m) != ST_FETCHING) {
        waiting = false;
        if (m_gen(m) != gen || m_rc(m) == 0) raise_error(c, E_STATE, ((uint64_t)idx << 8) | gen);
      }
    }
    if (ballot(waiting) && !sp.step(c, wi(W_TICKET, rdlane(idx, ffs64(ballot(waiting)))))) {
      okay = false;
      break;
    }
  }
  fence_acq();
  if (i < n) {
    ptrs[i] = (okay && st == TK_OK) ? (void*)(line_ptr(c, idx) + ((uint64_t)boff << 12)) : nullptr;
  }
  const uint64_t ne = __popcll(ballot(i < n && st == TK_EAGAIN));
  if (lane() == 0 && ne) add_rlx(counter(c, C_AUX0), ne);
  user_wave_done(c, li);
}

__global__ __launch_bounds__(WG) void k_release(dev_ctx c, launch_t li, const agile_ticket* tickets,
                                                uint32_t n) {
  user_wave_begin();
  const uint32_t uw = blockIdx.x * WPB + threadIdx.x / 64;
  const uint64_t i = (uint64_t)uw * 64 + lane();
  if (i < n) {
    const uint64_t t = tickets[i];
    const uint32_t idx = (uint32_t)t;
    if (((t >> 40) & 0xFF) == TK_OK && idx < c.num_lines) add_rel(c.meta + idx, (uint64_t)0 - RC_ONE);
  }
  user_wave_done(c, li);
}

// Flush: every DIRTY, unpinned line becomes WRITEBACK and gets one WRITE; the launch's
// service wavefronts drain them (WRITEBACK -> READY).  A pinned dirty line is an error.
__global__ __launch_bounds__(WG) void k_flush(dev_ctx c, launch_t li) {
  if (blockIdx.x < li.service_blocks) {
    run_service(c, li);
    return;
  }
  user_wave_begin();
  const uint32_t uw = (blockIdx.x - li.service_blocks) * WPB + threadIdx.x / 64;
  const uint32_t q = uw % c.num_qp;
  for (uint64_t base = (uint64_t)uw * 64; base < c.num_lines; base += (uint64_t)li.user_waves * 64) {
    const uint64_t i = base + lane();
    bool wb = false;
    uint32_t tag = 0;
    if (i < c.num_lines) {
      uint64_t m = ld_rlx(c.meta + i);
      if (m_state(m) == ST_DIRTY) {
        if (m_rc(m) != 0) {
          raise_error(c, E_STATE, i);
        } else if (cas(c.meta + i, m, (m & ~M_STATE) | ST_WRITEBACK)) {
          wb = true;
          tag = m_tag(m);
        } else {
          raise_error(c, E_STATE, i);
        }
      }
    }
    const uint64_t nw = __popcll(ballot(wb));
    if (lane() == 0) count(c, C_WB_FLUSH, nw);
    if (!submit_line(c, q, wb, OPC_WRITE, (uint32_t)i, tag)) break;
  }
  user_wave_done(c, li);
}

// Write-through of whole lines (Sec. 3.5's write through the cache: the caller's buffer
// may be reused once the call is done).  Lane i of a chunk takes lines[i]: the line is
// found or allocated without a READ (its whole content is replaced; a dirty victim is
// written back first), claimed by turning it WRITEBACK, filled from src by the whole
// wave and sent to its device as one WRITE; the completion leaves it READY (clean) with
// the new data.  A resident line is claimed only while no other write of it is in
// flight, and a wave never holds a claimed line while it waits for another one: each
// line is filled and submitted in the round that claimed it.  Lanes that found no
// evictable way retry once the wave's other writes are out.  Of lanes that name the
// same line, the highest writes it.
__global__ __launch_bounds__(WG) void k_write_lines(dev_ctx c, launch_t li, const uint64_t* lines, uint32_t n,
                                                    const uint8_t* src) {
  if (blockIdx.x < li.service_blocks) {
    run_service(c, li);
    return;
  }
  user_wave_begin();
  const uint32_t uw = (blockIdx.x - li.service_blocks) * WPB + threadIdx.x / 64;
  const uint32_t q = uw % c.num_qp;
  const uint64_t line_bytes = 1ull << c.line_shift;
  const uint64_t nlines = (c.store_blocks + c.blocks_per_line - 1) / c.blocks_per_line;
  for (uint64_t base = (uint64_t)uw * 64; base < n; base += (uint64_t)li.user_waves * 64) {
    const uint64_t i = base + lane();
    bool todo = i < n;
    uint32_t lid = 0;
    if (todo) {
      const uint64_t l = lines[i];
      if (l >= nlines) {
        raise_error(c, E_STATE, l);
        todo = false;
      }
      lid = (uint32_t)l;
    }
    spin_t sp;
    while (ballot(todo)) {
      chunk_t ch;
      ch.act = todo;
      ch.line_id = lid;
      ch.off = 0;
      if (!chunk_issue(c, ch, q, true, PIN_LINE, false, false)) goto out;
      const bool ok = ch.act && st_ok(ch.st);
      // source lane of each line: the highest lane of its leader's group
      uint32_t from = lane();
      for (uint64_t t = ballot(ok); t;) {
        const uint32_t ld = rdlane(ch.leader, ffs64(t));
        const uint64_t g = ballot(ok && ch.leader == ld);
        if (lane() == ld) from = 63 - __builtin_clzll(g);
        t &= ~g;
      }
      const bool lead = ok && ch.leader == lane();
      // claim READY / DIRTY (resident) or our own FETCHING (just allocated) ->
      // WRITEBACK; fill and submit what each round claimed
      bool claiming = lead;
      spin_t sc;
      while (ballot(claiming)) {
        bool got = false;
        if (claiming) {
          uint64_t m = ld_rlx(c.meta + ch.idx);
          const uint32_t st = m_state(m);
          const bool mine = st == ST_FETCHING && ch.st == A_MISS && m_gen(m) == ch.gen;
          if (m_tag(m) != ch.line_id) {
            raise_error(c, E_STATE, ch.idx);
            add_rel(c.meta + ch.idx, (uint64_t)0 - RC_ONE);
            claiming = false;
          } else if ((st == ST_READY || st == ST_DIRTY || mine) &&
                     cas(c.meta + ch.idx, m, (m & ~M_STATE) | ST_WRITEBACK)) {
            got = true;
            claiming = false;
          }
        }
        const uint64_t gm = ballot(got);
        if (gm) {
          // the last reader of the line's old content (the WRITE before ours) is done
          fence_acq();
          for (uint64_t t = gm; t; t &= t - 1) {
            const uint32_t l = ffs64(t);
            const uint64_t si = base + rdlane(from, l);
            const uint4* s4 = reinterpret_cast<const uint4*>(src + si * line_bytes);
            uint4* d4 = reinterpret_cast<uint4*>(line_ptr(c, rdlane(ch.idx, l)));
            for (uint64_t o = lane(); o < line_bytes / 16; o += 64) d4[o] = s4[o];
          }
          fence_rel();  // the line's data before the command that copies it out
          if (!submit_line(c, q, got, OPC_WRITE, ch.idx, ch.line_id)) goto out;
          // the WRITE is queued: the pin can go (a WRITEBACK line is never evicted)
          if (got) add_rel(c.meta + ch.idx, (uint64_t)0 - RC_ONE);
        }
        if (ballot(claiming) && !sc.step(c, wi(W_CLAIM, rdlane(ch.idx, ffs64(ballot(claiming)))))) goto out;
      }
      if (ch.act && ch.st != A_EAGAIN) todo = false;
      if (ballot(todo) && !sp.step(c, wi(W_WAY, rdlane(lid, ffs64(ballot(todo)))))) goto out;
    }
  }
out:
  user_wave_done(c, li);
}

// ---- reads into user buffers and the Share Table (Sec. 3.4.1, Listing 1's asyncRead)
// Share Table slot of block `blk` for a request whose buffer is `mine`: the first live
// holder of a block owns the slot and its buffer is the block's; later requests share
// that buffer (a holder count).  Returns 1 = owner, 2 = no slot along the probe (not
// registered), 3 = shared (`ptr` = the owner's buffer).  One lane.
__device__ __forceinline__ uint32_t share_acquire(const dev_ctx& c, uint64_t blk, uint64_t mine, uint64_t& ptr) {
  const uint64_t key = blk + 1;
  uint32_t h = (uint32_t)((blk * 0x9E3779B97F4A7C15ull) >> 40) & (SHARE_CAP - 1);
  for (uint32_t p = 0; p < SHARE_PROBES; ++p, h = (h + 1) & (SHARE_CAP - 1)) {
    uint64_t k = ld_rlx(c.share_key + h);
    if (k == 0) {
      uint64_t z = 0;
      k = cas(c.share_key + h, z, key) ? key : z;  // z holds the key that won the slot
    }
    if (k != key) continue;
    for (uint32_t spins = 0;; ++spins) {
      uint32_t r = __hip_atomic_load(c.share_refs + h, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
      if (r == SHARE_BUSY) {  // an owner is installing its buffer: a few stores away
        __builtin_amdgcn_s_sleep(1);
        if (spins > (1u << 20)) {
          raise_error(c, E_TIMEDOUT, wi(W_CLAIM, h));
          ptr = mine;
          return 2;
        }
        continue;
      }
      if (r == 0) {  // no live holder: become the owner
        if (cas(c.share_refs + h, r, SHARE_BUSY)) {
          st_rlx(c.share_buf + h, mine);
          __hip_atomic_store(c.share_refs + h, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
          ptr = mine;
          return 1;
        }
        continue;
      }
      if (cas(c.share_refs + h, r, r + 1)) {
        fence_acq();
        ptr = ld_rlx(c.share_buf + h);
        return 3;
      }
    }
  }
  ptr = mine;
  return 2;
}

// Copies 4 KiB from src to dst with the whole wave (64 lanes x 4 x 16 bytes).
__device__ __forceinline__ void copy_block_wave(const uint8_t* src, uint8_t* dst) {
  const uint4* s4 = reinterpret_cast<const uint4*>(src);
  uint4* d4 = reinterpret_cast<uint4*>(dst);
  uint4 v[4];
#pragma unroll
  for (uint32_t i = 0; i < 4; ++i) v[i] = s4[i * 64 + lane()];
#pragma unroll
  for (uint32_t i = 0; i < 4; ++i) d4[i * 64 + lane()] = v[i];
}

// Request i delivers block blocks[i] into buffer bufs[i] (device, 16-byte aligned), or,
// with sharing, points at the buffer of a live holder of the same block.  A resident
// block is copied at once; a block whose line is being filled puts its buffer on the
// line's pending list (the completion service copies it before the line turns READY), so
// the wave goes on to its next requests instead of waiting; a list found closed (the
// fill has landed) makes the wave copy the block itself once the line is READY.  Pins are
// held only while a wave copies or appends.  A set with no evictable way is retried with
// nothing held.
__global__ __launch_bounds__(WG) void k_async_issue(dev_ctx c, launch_t li, const uint64_t* blocks, uint32_t n,
                                                    void* const* bufs, void** ptrs, uint32_t* status, uint32_t share) {
  if (blockIdx.x < li.service_blocks) {
    run_service(c, li);
    return;
  }
  user_wave_begin();
  const uint32_t uw = (blockIdx.x - li.service_blocks) * WPB + threadIdx.x / 64;
  const uint32_t q = uw % c.num_qp;
  for (uint64_t base = (uint64_t)uw * 64; base < n; base += (uint64_t)li.user_waves * 64) {
    const uint64_t i = base + lane();
    bool todo = i < n;
    uint64_t blk = 0, dst = 0, ptr = 0;
    uint32_t st = AGILE_BUF_PRIVATE;
    if (todo) {
      blk = blocks[i];
      dst = (uint64_t)(uintptr_t)bufs[i];
      if (blk >= c.store_blocks || (dst & 15) || !dst) {
        raise_error(c, E_STATE, blk);
        todo = false;
      } else if (share) {
        st = share_acquire(c, blk, dst, ptr);
        if (st == AGILE_BUF_SHARED) todo = false;  // another holder's buffer has (or will have) it
      }
      if (st != AGILE_BUF_SHARED) ptr = dst;
    }
    const uint32_t boff = (uint32_t)((blk % c.blocks_per_line) << 12);
    spin_t sp;
    while (ballot(todo)) {
      chunk_t ch;
      ch.act = todo;
      ch.line_id = (uint32_t)(blk / c.blocks_per_line);
      ch.off = boff;
      if (!chunk_issue(c, ch, q, true, PIN_LINE)) goto out;
      const bool got = ch.act && st_ok(ch.st);
      // lines being filled: append to the pending list while still pinned (the pin keeps
      // the line from a new tenant, so the list appended to is this fill's)
      bool self = got && ch.st == A_HIT;
      if (got && ch.st != A_HIT) {
        const uint64_t e = add_rlx(counter(c, C_PEND), 1ull);
        if (e >= PEND_CAP) {
          self = true;  // no entry left: copy it ourselves
        } else {
          st_rlx(c.pend + 2 * e, dst);
          fence_rel();
          uint32_t h = ld_rlx(c.pend_head + ch.idx);
          for (;;) {
            if (h == PEND_CLOSED) {
              self = true;  // the fill has landed (or is being delivered): copy it ourselves
              break;
            }
            st_rlx(c.pend + 2 * e + 1, ((uint64_t)boff << 32) | h);
            fence_rel();
            if (cas(c.pend_head + ch.idx, h, (uint32_t)e)) break;
          }
        }
      }
      // copies by the wave itself: wait (per lane: the pin keeps the tenant) until the
      // line holds its data, then copy
      {
        bool waiting = self;
        spin_t sw;
        while (ballot(waiting)) {
          if (waiting) {
            const uint64_t m = ld_rlx(c.meta + ch.idx);
            if (m_state(m) != ST_FETCHING || m_tag(m) != ch.line_id || m_gen(m) != ch.gen) waiting = false;
          }
          if (ballot(waiting) && !sw.step(c, wi(W_FILL, rdlane(ch.idx, ffs64(ballot(waiting)))))) goto out;
        }
        fence_acq();
      }
      for (uint64_t t = ballot(self); t; t &= t - 1) {
        const uint32_t l = ffs64(t);
        copy_block_wave(line_ptr(c, rdlane(ch.idx, l)) + rdlane(ch.off, l),
                        reinterpret_cast<uint8_t*>((uintptr_t)rdlane64(dst, l)));
      }
      chunk_release(c, ch, false);
      if (got) todo = false;
      if (ballot(todo) && !sp.step(c, wi(W_WAY, rdlane(ch.line_id, ffs64(ballot(todo)))))) goto out;
    }
    if (i < n) {
      ptrs[i] = (void*)(uintptr_t)ptr;
      status[i] = st;
    }
  }
out:
  user_wave_done(c, li);
}

// Drops Share Table holds: request i's hold of block blocks[i] if status[i] says it
// has one (owner or sharer).  Not a service kernel.
__global__ void k_share_release(dev_ctx c, const uint64_t* blocks, const uint32_t* status, uint32_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t st = status[i];
  if (st != AGILE_BUF_OWNER && st != AGILE_BUF_SHARED) return;
  const uint64_t blk = blocks[i], key = blk + 1;
  uint32_t h = (uint32_t)((blk * 0x9E3779B97F4A7C15ull) >> 40) & (SHARE_CAP - 1);
  for (uint32_t p = 0; p < SHARE_PROBES; ++p, h = (h + 1) & (SHARE_CAP - 1)) {
    if (ld_rlx(c.share_key + h) != key) continue;
    uint32_t r = ld_rlx(c.share_refs + h);
    for (;;) {
      if (r == 0 || r == SHARE_BUSY) {
        raise_error(c, E_STATE, blk);  // released more often than held
        return;
      }
      if (cas(c.share_refs + h, r, r - 1)) return;
    }
  }
  raise_error(c, E_STATE, blk);
}

// The owner propagates its buffer's changes (Sec. 3.4.1): block blocks[i] takes the
// 4 KiB at srcs[i] inside its cache line (read first on a miss), which becomes MODIFIED
// and is written back on eviction or at agile_flush.
__global__ __launch_bounds__(WG) void k_buf_writeback(dev_ctx c, launch_t li, const uint64_t* blocks, uint32_t n,
                                                      const void* const* srcs) {
  if (blockIdx.x < li.service_blocks) {
    run_service(c, li);
    return;
  }
  user_wave_begin();
  const uint32_t uw = (blockIdx.x - li.service_blocks) * WPB + threadIdx.x / 64;
  const uint32_t q = uw % c.num_qp;
  for (uint64_t base = (uint64_t)uw * 64; base < n; base += (uint64_t)li.user_waves * 64) {
    const uint64_t i = base + lane();
    bool todo = i < n;
    uint64_t blk = 0, src = 0;
    if (todo) {
      blk = blocks[i];
      src = (uint64_t)(uintptr_t)srcs[i];
      if (blk >= c.store_blocks || (src & 15) || !src) {
        raise_error(c, E_STATE, blk);
        todo = false;
      }
    }
    // lanes naming the same line take turns: one lane per distinct line per round
    spin_t sp;
    while (ballot(todo)) {
      chunk_t ch;
      ch.act = todo;
      ch.line_id = (uint32_t)(blk / c.blocks_per_line);
      ch.off = (uint32_t)((blk % c.blocks_per_line) << 12);
      dedup(ch, todo);
      const bool first = todo && ch.leader == lane();
      ch.act = first;
      if (!chunk_issue(c, ch, q, true, PIN_LINE)) goto out;
      if (!chunk_wait(c, ch)) goto out;
      const bool got = first && st_ok(ch.st);
      {
        // a line being written back (an eviction that chose it before our pin) is
        // modified only once that write has landed
        bool wbw = got;
        spin_t sw;
        while (ballot(wbw)) {
          if (wbw && m_state(ld_rlx(c.meta + ch.idx)) != ST_WRITEBACK) wbw = false;
          if (ballot(wbw) && !sw.step(c, wi(W_WB, rdlane(ch.idx, ffs64(ballot(wbw)))))) goto out;
        }
        fence_acq();
      }
      for (uint64_t t = ballot(got); t; t &= t - 1) {
        const uint32_t l = ffs64(t);
        copy_block_wave(reinterpret_cast<const uint8_t*>((uintptr_t)rdlane64(src, l)),
                        line_ptr(c, rdlane(ch.idx, l)) + rdlane(ch.off, l));
      }
      if (got) {
        uint64_t mv = ld_rlx(c.meta + ch.idx);
        while (m_state(mv) == ST_READY) {
          if (cas(c.meta + ch.idx, mv, mv + 1ull)) break;  // READY -> MODIFIED
        }
      }
      chunk_release(c, ch, true);
      if (got) todo = false;
      if (ballot(todo) && !ballot(got) && !sp.step(c, wi(W_WAY, rdlane(ch.line_id, ffs64(ballot(todo)))))) goto out;
    }
  }
out:
  user_wave_done(c, li);
}

__global__ __launch_bounds__(WG) void k_invalidate(dev_ctx c, launch_t li) {
  user_wave_begin();
  const uint32_t uw = blockIdx.x * WPB + threadIdx.x / 64;
  const uint64_t i = (uint64_t)uw * 64 + lane();
  if (i < c.num_lines) {
    uint64_t m = ld_rlx(c.meta + i);
    const uint32_t st = m_state(m);
    if (st == ST_READY && m_rc(m) == 0) {
      if (!cas(c.meta + i, m, m & ~(M_STATE | M_REF))) raise_error(c, E_STATE, i);
    } else if (st != ST_INVALID) {
      raise_error(c, E_STATE, i);
    }
  }
  // clock hands back to way 0 so that a cold cache replays like a fresh one
  for (uint64_t s = i; s < c.num_sets; s += (uint64_t)li.user_waves * 64) st_rlx(c.hand + s, 0u);
  user_wave_done(c, li);
}

// Serialized request trace for the clock-policy comparison: lane 0 of one wave acquires
// line ids one at a time (write requests turn the line DIRTY), recording hit/miss and way.
__global__ __launch_bounds__(WG) void k_trace(dev_ctx c, launch_t li, const uint64_t* lines,
                                              const uint8_t* writes, uint64_t n, uint8_t* hit,
                                              int32_t* way) {
  if (blockIdx.x < li.service_blocks) {
    run_service(c, li);
    return;
  }
  user_wave_begin();
  const uint32_t uw = (blockIdx.x - li.service_blocks) * WPB + threadIdx.x / 64;
  if (uw == 0) {
    for (uint64_t i = 0; i < n; ++i) {
      chunk_t ch;
      ch.act = lane() == 0;
      ch.line_id = (uint32_t)lines[i];
      ch.off = 0;
      const bool w = writes && writes[i];
      spin_t sp;
      for (;;) {
        if (!chunk_issue(c, ch, 0, true, PIN_LINE)) goto out;
        if (!chunk_wait(c, ch)) goto out;
        if (rdlane(ch.st, 0) != A_EAGAIN) break;
        if (!sp.step(c, wi(W_WAY, 0))) goto out;
      }
      if (lane() == 0) {
        hit[i] = (ch.st == A_MISS) ? 0 : 1;
        way[i] = (int32_t)(ch.idx % c.assoc);
        if (w) {
          uint64_t m = ld_rlx(c.meta + ch.idx);
          while (m_state(m) == ST_READY) {
            if (cas(c.meta + ch.idx, m, m + 1ull)) break;  // READY -> DIRTY
          }
        }
      }
      chunk_release(c, ch, w);
    }
  }
out:
  user_wave_done(c, li);
}

// ---- embedding-bag backward fused with SGD (write path)
struct bwd_args {
  const int64_t* idx;
  const int64_t* off;
  const float* grad;      // [B*T, dim] upstream gradient of the pooled output
  uint64_t* keys;         // (global row << 32 | lookup position), sorted
  uint32_t* bagid;        // bag of each lookup position
  uint32_t* heads;        // first sorted position of every distinct row (unordered)
  uint32_t* ctr;          // [0] = number of heads, [1] = group counter
  uint64_t n, nbags, rows, base_off;
  uint32_t T, dim, row_bytes;
  float lr;
};

__global__ void k_bwd_keys(bwd_args a, uint64_t* keys_in) {
  const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= a.nbags) return;
  const uint64_t t = g % a.T;
  for (int64_t j = a.off[g]; j < a.off[g + 1]; ++j) {
    keys_in[j] = ((t * a.rows + (uint64_t)a.idx[j]) << 32) | (uint64_t)j;
    a.bagid[j] = (uint32_t)g;
  }
}

__global__ void k_bwd_heads(bwd_args a) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  if (i == 0 || (a.keys[i] >> 32) != (a.keys[i - 1] >> 32)) {
    const uint32_t k = atomicAdd(a.ctr, 1u);
    a.heads[k] = (uint32_t)i;
  }
}

// One user wave takes 64 distinct rows at a time: pins their lines for writing, sums each
// row's upstream gradients over its occurrences in ascending lookup position (fp32, from
// +0.0f), applies w = fmaf(-lr, g, w) in the cached line, marks the line MODIFIED and
// unpins it with release ordering.  A MODIFIED line is written back when the clock evicts
// it or at flush (Sec. 3.4, case d).
template <int VPL>
__device__ __forceinline__ void bwd_wave(const dev_ctx& c, const bwd_args& a, uint32_t uw) {
  const uint32_t q = uw % c.num_qp;
  const uint32_t nheads = ld_rlx(a.ctr);
  const uint32_t d0 = lane() * VPL;
  const bool mine = d0 < a.dim;
  for (;;) {
    uint32_t gidx = 0;
    if (lane() == 0) gidx = add_rlx(a.ctr + 1, 1u);
    gidx = rdlane(gidx, 0);
    const uint64_t base = (uint64_t)gidx * 64;
    if (base >= nheads) break;
    bool todo = base + lane() < nheads;
    uint32_t start = 0;
    uint64_t row = 0;
    if (todo) {
      start = a.heads[base + lane()];
      row = a.keys[start] >> 32;
    }
    spin_t sp;
    while (ballot(todo)) {
      chunk_t ch;
      ch.act = todo;
      if (todo) {
        const uint64_t byte = a.base_off + row * a.row_bytes;
        ch.line_id = (uint32_t)(byte >> c.line_shift);
        ch.off = (uint32_t)(byte & ((1ull << c.line_shift) - 1));
      }
      if (!chunk_issue(c, ch, q, true, PIN_LINE)) return;
      // No acquire (it would drop the whole L2 of the XCD): within a launch a row has one
      // writer, this wave, so its current value is the one the fill (or an earlier
      // launch) left, read below with device-coherent loads past any stale L2 copy.
      if (!chunk_wait(c, ch, false)) return;
      // a line pinned while its earlier write-back was in flight: wait for it to finish
      // (the write-back only reads the line)
      bool wbw = ch.act && st_ok(ch.st) && ch.leader == lane();
      while (ballot(wbw)) {
        if (wbw && m_state(ld_rlx(c.meta + ch.idx)) != ST_WRITEBACK) wbw = false;
        if (ballot(wbw) && !sp.step(c, wi(W_WB, rdlane(ch.idx, ffs64(ballot(wbw)))))) return;
      }
      const uint64_t okm = ballot(ch.act && st_ok(ch.st));
      for (uint64_t m = okm; m; m &= m - 1) {
        const uint32_t k = ffs64(m);
        const uint32_t s0 = rdlane(start, k);
        const uint64_t r = rdlane64(row, k);
        // segment end: first sorted position past s0 with another row
        uint64_t e = s0 + 1;
        for (;;) {
          const uint64_t i = e + lane();
          const bool same = i < a.n && (a.keys[i] >> 32) == r;
          const uint64_t b = ballot(same);
          const uint32_t run = (~b == 0ull) ? 64u : ffs64(~b);
          e += run;
          if (run < 64) break;
        }
        float acc[VPL];
#pragma unroll
        for (int v = 0; v < VPL; ++v) acc[v] = 0.0f;
        for (uint64_t i = s0; i < e; ++i) {
          const uint32_t j = (uint32_t)a.keys[i];
          const uint32_t gb = a.bagid[j];
          if (mine) {
            const float* gp = a.grad + (uint64_t)gb * a.dim + d0;
#pragma unroll
            for (int v = 0; v < VPL; ++v) acc[v] = acc[v] + gp[v];
          }
        }
        const uint32_t idx = rdlane(ch.idx, k);
        const uint32_t off = rdlane(ch.off, k);
        float* w = reinterpret_cast<float*>(line_ptr(c, idx) + off) + d0;
        if (mine) {
          float wv[VPL];
          ld_row<VPL>(w, wv);
#pragma unroll
          for (int v = 0; v < VPL; ++v) w[v] = __builtin_fmaf(-a.lr, acc[v], wv[v]);
        }
      }
      // mark the written lines MODIFIED (leaders), then unpin with release ordering
      if (ch.act && st_ok(ch.st) && ch.leader == lane()) {
        uint64_t mv = ld_rlx(c.meta + ch.idx);
        while (m_state(mv) == ST_READY) {
          if (cas(c.meta + ch.idx, mv, mv + 1ull)) break;  // READY -> DIRTY
        }
      }
      if (lane() == 0) wcount(WS_WROWS, __popcll(okm));
      chunk_release(c, ch, true);
      if (okm && ((okm >> lane()) & 1ull)) todo = false;
      if (ballot(todo) && !okm) {
        if (!sp.step(c, wi(W_WAY, gidx))) return;
      }
    }
  }
}

// With a next batch (p.nbags), the first p.waves waves first prefetch its lines (the
// next step's forward then finds them resident) and then join the others, which take
// the distinct rows' groups from a counter meanwhile.
template <int VPL>
__global__ __launch_bounds__(WG) void k_bwd_sgd(dev_ctx c, launch_t li, bwd_args a, pf_args p) {
  if (blockIdx.x < li.service_blocks) {
    run_service(c, li);
    return;
  }
  user_wave_begin();
  const uint32_t uw = (blockIdx.x - li.service_blocks) * WPB + threadIdx.x / 64;
  if (!(uw < p.waves && p.nbags) || prefetch_wave(c, p, uw)) bwd_wave<VPL>(c, a, uw);
  user_wave_done(c, li);
}

// ---- graph workloads over a CSR graph held in the store (row_ptr int64, col int32, val fp32)
struct csr_t {
  uint64_t V, E, rp_off, col_off, val_off;
};

// Reads one aligned 4- or 8-byte word per active lane from the store through the cache,
// optimistically: lines are not pinned unless this wave's own miss filled them, and the
// line's tag and generation are re-checked after the load.  Lanes whose line changed, or
// whose set had no evictable way, retry while holding nothing.
// `drop` runs before the wave backs off to retry: a caller that holds pins of its own
// (a prefetch) releases them there, so it never waits for a way while pinning lines.
template <typename T, typename Drop>
__device__ __forceinline__ bool cached_read(const dev_ctx& c, uint32_t q, bool act, uint64_t byte, T& out,
                                            Drop&& drop) {
  bool todo = act;
  spin_t sp;
  while (ballot(todo)) {
    chunk_t ch;
    ch.act = todo;
    if (todo) {
      ch.line_id = (uint32_t)(byte >> c.line_shift);
      ch.off = (uint32_t)(byte & ((1ull << c.line_shift) - 1));
    }
    if (!chunk_issue(c, ch, q, true, PIN_NONE, false)) return false;
    if (!chunk_wait(c, ch, false)) return false;
    const bool got = todo && st_ok(ch.st);
    T v = 0;
    if (got) v = ld_rlx(reinterpret_cast<const T*>(line_ptr(c, ch.idx) + ch.off));
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");  // the load has completed
    bool ok = false;
    if (got) ok = ch.pinned || line_still_valid(c, ch.idx, ch.line_id, ch.gen);
    if (ok) out = v;
    chunk_release(c, ch, false);
    if (ok) todo = false;
    if (ballot(todo) && !ballot(ok)) {
      drop();
      if (!sp.step(c, wi(W_WAY, 0))) return false;
    }
  }
  return true;
}
template <typename T>
__device__ __forceinline__ bool cached_read(const dev_ctx& c, uint32_t q, bool act, uint64_t byte, T& out) {
  return cached_read<T>(c, q, act, byte, out, [] {});
}

// A store word for the graph kernels: through the cache, or, when `img` is set, straight
// from a copy of the store image resident in HBM (the kernel-only baseline of Sec. 4.5,
// where the graph kernels run with no cache, queue or service in the way).
template <typename T>
__device__ __forceinline__ bool graph_read(const dev_ctx& c, uint32_t q, const uint8_t* img, bool act, uint64_t byte,
                                           T& out) {
  if (img) {
    if (act) out = *reinterpret_cast<const T*>(img + byte);
    return true;
  }
  return cached_read<T>(c, q, act, byte, out);
}

struct bfs_args {
  csr_t g;
  const uint8_t* img;  // resident copy of the store image (NULL: read through the cache)
  const int32_t* F;   // frontier
  uint32_t nF;
  uint64_t* cs;       // compacted: first edge of each frontier vertex with edges
  uint64_t* cd;       // compacted: its out-degree
  uint64_t* co;       // exclusive prefix sums of cd
  uint32_t* ctr;      // [0] compacted count, [1] next-frontier count, [2] work counter
  int32_t* N;         // next frontier
  int32_t* level;
  int32_t L;          // current level
  uint32_t nC;
  uint64_t Et;        // edges out of the frontier
};

// Level step 1: each frontier vertex reads its row_ptr pair through the cache; vertices
// with edges are compacted (order is irrelevant: levels do not depend on it).
__global__ __launch_bounds__(WG) void k_bfs_front(dev_ctx c, launch_t li, bfs_args a) {
  if (blockIdx.x < li.service_blocks) {
    run_service(c, li);
    return;
  }
  user_wave_begin();
  const uint32_t uw = (blockIdx.x - li.service_blocks) * WPB + threadIdx.x / 64;
  const uint32_t q = uw % c.num_qp;
  for (uint64_t base = (uint64_t)uw * 64; base < a.nF; base += (uint64_t)li.user_waves * 64) {
    const bool act = base + lane() < a.nF;
    const uint64_t v = act ? (uint64_t)a.F[base + lane()] : 0;
    const uint64_t b0 = a.g.rp_off + 8 * v;
    int64_t s0 = 0, s1 = 0;
    if (!graph_read<int64_t>(c, q, a.img, act, b0, s0)) break;
    if (!graph_read<int64_t>(c, q, a.img, act, b0 + 8, s1)) break;
    const bool has = act && s1 > s0;
    const uint64_t hm = ballot(has);
    uint32_t pos = 0;
    if (lane() == 0 && hm) pos = atomicAdd(a.ctr, (uint32_t)__popcll(hm));
    pos = rdlane(pos, 0) + mbcnt(hm);
    if (has) {
      a.cs[pos] = (uint64_t)s0;
      a.cd[pos] = (uint64_t)(s1 - s0);
    }
  }
  user_wave_done(c, li);
}

// Level step 2: the frontier's edges, flattened by the prefix sums, are split into chunks
// of 1024 so that a hub vertex is spread over many waves.  Each lane reads one col entry
// through the cache and claims unvisited vertices with a CAS on level[].
__global__ __launch_bounds__(WG) void k_bfs_edges(dev_ctx c, launch_t li, bfs_args a) {
  if (blockIdx.x < li.service_blocks) {
    run_service(c, li);
    return;
  }
  user_wave_begin();
  const uint32_t uw = (blockIdx.x - li.service_blocks) * WPB + threadIdx.x / 64;
  const uint32_t q = uw % c.num_qp;
  for (;;) {
    uint32_t g = 0;
    if (lane() == 0) g = atomicAdd(a.ctr + 2, 1u);
    g = rdlane(g, 0);
    const uint64_t e0 = (uint64_t)g * 1024;
    if (e0 >= a.Et) break;
    const uint64_t e1 = (e0 + 1024 < a.Et) ? e0 + 1024 : a.Et;
    // vertex holding edge e0: 64-ary search over co (wave parallel)
    uint64_t lo = 0, hi = a.nC;  // invariant: co[lo] <= e0 < co[hi] (co[nC] = Et)
    while (hi - lo > 1) {
      const uint64_t step = (hi - lo + 63) / 64;
      const uint64_t p = lo + (uint64_t)lane() * step;
      const bool le = p < hi && a.co[p] <= e0;
      const uint64_t m = ballot(le);
      const uint32_t k = 63 - __builtin_clzll(m);  // last lane with co[p] <= e0
      const uint64_t nlo = lo + (uint64_t)k * step;
      const uint64_t nhi = (nlo + step < hi) ? nlo + step : hi;
      lo = nlo;
      hi = nhi;
    }
    uint64_t i = lo;
    for (uint64_t e = e0; e < e1; e += 64) {
      const uint64_t my = e + lane();
      const bool act = my < e1;
      // window of 64 vertices from i: every compacted vertex has >= 1 edge, so it covers
      const uint64_t wi = i + lane();
      const uint64_t wco = wi < a.nC ? a.co[wi] : ~0ull;
      uint32_t k = 0;
#pragma unroll
      for (uint32_t st = 32; st; st >>= 1) {
        const uint64_t cand = (uint64_t)shfl32((uint32_t)(wco >> 32), k + st) << 32 |
                              shfl32((uint32_t)wco, k + st);
        if (k + st < 64 && cand <= my) k += st;
      }
      const uint64_t vo = (uint64_t)shfl32((uint32_t)(wco >> 32), k) << 32 | shfl32((uint32_t)wco, k);
      const uint64_t vs = act ? a.cs[i + k] : 0;
      const uint64_t pos = vs + (my - vo);
      int32_t u = 0;
      if (!graph_read<int32_t>(c, q, a.img, act, a.g.col_off + 4 * pos, u)) goto done;
      bool added = false;
      if (act && (uint64_t)u < a.g.V) {
        if (__hip_atomic_load(a.level + u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == -1) {
          int32_t expect = -1;
          added = __hip_atomic_compare_exchange_strong(a.level + u, &expect, a.L + 1, __ATOMIC_RELAXED,
                                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      const uint64_t am = ballot(added);
      uint32_t pos2 = 0;
      if (lane() == 0 && am) pos2 = atomicAdd(a.ctr + 1, (uint32_t)__popcll(am));
      pos2 = rdlane(pos2, 0) + mbcnt(am);
      if (added) a.N[pos2] = u;
      // keep i = the vertex of the next step's first edge (e + 64)
      const uint32_t kl = rdlane(k, 63);
      uint64_t nxt = ~0ull;
      if (lane() == 0 && i + kl + 1 < a.nC) nxt = a.co[i + kl + 1];
      nxt = rdlane64(nxt, 0);
      i += kl + (nxt == e + 64 ? 1u : 0u);
    }
  }
done:
  user_wave_done(c, li);
}

// SpMV: a wave takes 64 consecutive rows, one per lane, and folds each row in CSR order,
// acc = fmaf(val[k], x[col[k]], acc) from +0.0f (the same order as the plain definition).
// The rows' edges are walked in windows of 2048: the window's col and val lines are pinned
// for the window and their indices kept in LDS, so lanes with long rows walk them freely.
struct spmv_args {
  csr_t g;
  const uint8_t* img;  // resident copy of the store image (NULL: read through the cache)
  const float* x;
  float* y;
  uint32_t active;  // user waves that take work
};

// Edges per pinned window: col and val each get eight line slots; a window of
// (L - 1) * line_bytes / 4 edges spans at most L lines of either array, and with
// L <= the number of sets those lines fall in distinct sets.
__device__ __forceinline__ uint64_t spmv_window(const dev_ctx& c) {
  const uint64_t L = c.num_sets < 8 ? (c.num_sets > 2 ? c.num_sets : 2) : 8;
  return ((L - 1) << c.line_shift) / 4;
}

// Lines of col[p0, p1) and val[p0, p1) requested ahead of their window (the asynchronous
// pattern of Sec. 4.2 applied to the edge stream): a line this wave claims stays pinned
// until the window that needs it has been pinned, and the request is never waited for.
struct spmv_pref {
  chunk_t ch;
  bool held;
};
__device__ __forceinline__ void spmv_drop(const dev_ctx& c, spmv_pref& pf) {
  if (pf.held) chunk_release(c, pf.ch, false);
  pf.held = false;
}
__device__ __forceinline__ bool spmv_prefetch(const dev_ctx& c, uint32_t q, const spmv_args& a, uint64_t p0,
                                              uint64_t p1, spmv_pref& pf) {
  pf.held = false;
  if (p0 >= p1) return true;
  const uint32_t lc0 = (uint32_t)((a.g.col_off + 4 * p0) >> c.line_shift);
  const uint32_t lv0 = (uint32_t)((a.g.val_off + 4 * p0) >> c.line_shift);
  const uint32_t nc = (uint32_t)((a.g.col_off + 4 * p1 - 1) >> c.line_shift) - lc0 + 1;
  const uint32_t nv = (uint32_t)((a.g.val_off + 4 * p1 - 1) >> c.line_shift) - lv0 + 1;
  pf.ch.act = lane() < nc || (lane() >= 8 && lane() < 8 + nv);
  pf.ch.line_id = lane() < 8 ? lc0 + lane() : lv0 + (lane() - 8);
  pf.ch.off = 0;
  if (!chunk_issue(c, pf.ch, q, true, PIN_NONE)) return false;
  pf.held = true;
  return true;
}

// Pins the lines that hold col[w0, w1) and val[w0, w1) (one line per lane, PIN_LINE) and
// publishes their cache indices in win[0, 8) (col) and win[8, 16) (val).  A set without
// an evictable way makes the wave drop everything, its prefetch included, and retry while
// holding nothing.
__device__ __forceinline__ bool spmv_pin(const dev_ctx& c, uint32_t q, const spmv_args& a, uint64_t w0,
                                         uint64_t w1, uint32_t* win, uint32_t& lc0, uint32_t& lv0,
                                         chunk_t& ch, spmv_pref& pf) {
  const uint64_t cb0 = a.g.col_off + 4 * w0, cb1 = a.g.col_off + 4 * w1 - 1;
  const uint64_t vb0 = a.g.val_off + 4 * w0, vb1 = a.g.val_off + 4 * w1 - 1;
  lc0 = (uint32_t)(cb0 >> c.line_shift);
  lv0 = (uint32_t)(vb0 >> c.line_shift);
  const uint32_t nc = (uint32_t)(cb1 >> c.line_shift) - lc0 + 1;
  const uint32_t nv = (uint32_t)(vb1 >> c.line_shift) - lv0 + 1;
  const bool todo = lane() < nc || (lane() >= 8 && lane() < 8 + nv);
  const uint32_t want = lane() < 8 ? lc0 + lane() : lv0 + (lane() - 8);
  spin_t sp;
  for (;;) {
    ch.act = todo;
    ch.line_id = want;
    ch.off = 0;
    if (!chunk_issue(c, ch, q, true, PIN_LINE)) return false;
    if (ballot(ch.act && ch.st == A_EAGAIN)) {
      chunk_release(c, ch, false);
      spmv_drop(c, pf);
      if (!sp.step(c, wi(W_WAY, 0))) return false;
      continue;
    }
    // no acquire (an agent-scope acquire drops the whole L2 of the XCD): the window's
    // lines are pinned, and their data is read with device-coherent loads issued after
    // the fill was observed
    if (!chunk_wait(c, ch, false)) return false;
    break;
  }
  if (todo) win[lane() < 8 ? lane() : 8 + (lane() - 8)] = ch.idx;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  return true;
}

struct spmv_edge {
  int32_t col;
  float val;
};
__device__ __forceinline__ spmv_edge spmv_load(const dev_ctx& c, const spmv_args& a, const uint32_t* win,
                                               uint32_t lc0, uint32_t lv0, uint64_t k) {
  const uint32_t lmask = (1u << c.line_shift) - 1;
  const uint64_t cb = a.g.col_off + 4 * k, vb = a.g.val_off + 4 * k;
  const uint32_t ci = win[(uint32_t)(cb >> c.line_shift) - lc0];
  const uint32_t vi = win[8 + (uint32_t)(vb >> c.line_shift) - lv0];
  spmv_edge e;
  e.col = (int32_t)ld_rlx(reinterpret_cast<const uint32_t*>(line_ptr(c, ci) + (cb & lmask)));
  e.val = __uint_as_float(ld_rlx(reinterpret_cast<const uint32_t*>(line_ptr(c, vi) + (vb & lmask))));
  return e;
}
__device__ __forceinline__ float spmv_x(const spmv_args& a, int32_t col) {
  return ((uint64_t)(uint32_t)col < a.g.V) ? a.x[col] : 0.0f;
}

// The rows of a wave's group (lane r holds row r's edge range [rs, re), the group's
// edges are [e0, e1)) are folded edge-parallel: the lanes load 64 consecutive edges at a
// time (four groups in flight: col and val from the pinned window, then x[col]) and the
// wave walks them in CSR order through lane reads, closing a row when its end is reached.
// Each row's result is therefore the fmaf chain of its edges in order, and the memory
// work per edge is the same for hub rows and for short ones.  Returns row r's value in
// lane r.
__device__ __forceinline__ bool spmv_group(const dev_ctx& c, uint32_t q, const spmv_args& a, uint32_t* win,
                                           uint64_t re, uint32_t nr, uint64_t e0, uint64_t e1, uint64_t pend,
                                           spmv_pref& pf, float& yv) {
  const uint64_t W = spmv_window(c);
  uint32_t r = 0;                  // current row (uniform)
  uint64_t er = rdlane64(re, 0);   // its end
  float acc = 0.0f;
  yv = 0.0f;
  for (uint64_t w0 = e0; w0 < e1; w0 += W) {
    const uint64_t w1 = (w0 + W < e1) ? w0 + W : e1;
    uint32_t lc0 = 0, lv0 = 0;
    chunk_t ch;
    ch.act = false;
    const uint64_t t_pin = now();
    uint64_t t_cons = t_pin;
    if (!a.img) {
      if (!spmv_pin(c, q, a, w0, w1, win, lc0, lv0, ch, pf)) return false;
      const uint64_t t_pre = wtick(c, WS_T_WAIT, t_pin);
      // this window is pinned: drop the request that brought it, and ask for the next one
      // (up to `pend`, the end of the wave's run of groups) before computing on this one
      spmv_drop(c, pf);
      if (!spmv_prefetch(c, q, a, w1, (w1 + W < pend) ? w1 + W : pend, pf)) return false;
      t_cons = wtick(c, WS_T_ISSUE, t_pre);
    }
    for (uint64_t k0 = w0; k0 < w1; k0 += 256) {
      float v[4], xv[4];
      int32_t col[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint64_t k = k0 + 64 * u + lane();
        col[u] = -1;
        v[u] = 0.0f;
        if (k < w1) {
          if (a.img) {
            col[u] = *reinterpret_cast<const int32_t*>(a.img + a.g.col_off + 4 * k);
            v[u] = *reinterpret_cast<const float*>(a.img + a.g.val_off + 4 * k);
          } else {
            const spmv_edge e = spmv_load(c, a, win, lc0, lv0, k);
            col[u] = e.col;
            v[u] = e.val;
          }
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) xv[u] = col[u] >= 0 ? spmv_x(a, col[u]) : 0.0f;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint64_t base = k0 + 64 * u;
        if (base >= w1) break;
        const uint32_t n = (w1 - base) < 64 ? (uint32_t)(w1 - base) : 64u;
        for (uint32_t j = 0; j < n; ++j) {
          while (base + j >= er) {  // row r is complete (rows without edges close at once)
            if (lane() == r) yv = acc;
            acc = 0.0f;
            ++r;
            er = rdlane64(re, r);
          }
          acc = __builtin_fmaf(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(v[u]), j)),
                               __int_as_float(__builtin_amdgcn_readlane(__float_as_int(xv[u]), j)), acc);
        }
      }
    }
    if (!a.img) {
      __builtin_amdgcn_wave_barrier();
      chunk_release(c, ch, false);
    }
    wtick(c, WS_T_CONSUME, t_cons);
  }
  // the row being folded when the edges ran out; the rows after it have no edges
  if (r < nr && lane() == r) yv = acc;
  return true;
}

// Groups of 64 rows taken per grab: a wave streams through their edges in order, so the
// next window to prefetch is the one after the current.
constexpr uint64_t SPMV_RUN = 16;

__global__ __launch_bounds__(WG) void k_spmv(dev_ctx c, launch_t li, spmv_args a) {
  __shared__ uint32_t win[WPB][16];
  if (blockIdx.x < li.service_blocks) {
    run_service(c, li);
    return;
  }
  user_wave_begin();
  const uint32_t wv = threadIdx.x / 64;
  const uint32_t uw = (blockIdx.x - li.service_blocks) * WPB + wv;
  const uint32_t q = uw % c.num_qp;
  spmv_pref pf;
  pf.held = false;
  for (;;) {
    if (uw >= a.active) break;
    uint64_t gi = 0;
    if (lane() == 0) gi = add_rlx(counter(c, C_WORK), 1ull);
    gi = rdlane64(gi, 0);
    const uint64_t rr0 = gi * 64 * SPMV_RUN;
    if (rr0 >= a.g.V) break;
    const uint64_t rr1 = (a.g.V - rr0) < 64 * SPMV_RUN ? a.g.V : rr0 + 64 * SPMV_RUN;
    auto drop = [&] { spmv_drop(c, pf); };
    int64_t pend = 0;
    if (a.img) {
      if (lane() == 0) pend = *reinterpret_cast<const int64_t*>(a.img + a.g.rp_off + 8 * rr1);
    } else if (!cached_read<int64_t>(c, q, lane() == 0, a.g.rp_off + 8 * rr1, pend, drop)) {
      goto done;
    }
    pend = (int64_t)rdlane64((uint64_t)pend, 0);
    for (uint64_t r0 = rr0; r0 < rr1; r0 += 64) {
      const uint32_t nr = (uint32_t)((rr1 - r0) < 64 ? (rr1 - r0) : 64);
      const bool act = lane() < nr;
      int64_t rs = 0, rend = 0;
      const uint64_t t_desc = now();
      if (a.img) {
        if (act) rs = *reinterpret_cast<const int64_t*>(a.img + a.g.rp_off + 8 * (r0 + lane()));
        if (lane() == 0) rend = *reinterpret_cast<const int64_t*>(a.img + a.g.rp_off + 8 * (r0 + nr));
      } else {
        if (!cached_read<int64_t>(c, q, act, a.g.rp_off + 8 * (r0 + lane()), rs, drop)) goto done;
        if (!cached_read<int64_t>(c, q, lane() == 0, a.g.rp_off + 8 * (r0 + nr), rend, drop)) goto done;
      }
      wtick(c, WS_T_DESC, t_desc);
      rend = (int64_t)rdlane64((uint64_t)rend, 0);
      int64_t re = (int64_t)shfl64((uint64_t)rs, (lane() + 1) & 63);
      if (lane() == nr - 1) re = rend;
      if (!act) re = rend;
      float yv;
      if (!spmv_group(c, q, a, win[wv], (uint64_t)re, nr, rdlane64((uint64_t)rs, 0), (uint64_t)rend,
                      (uint64_t)pend, pf, yv))
        goto done;
      if (act) a.y[r0 + lane()] = yv;
    }
    spmv_drop(c, pf);
  }
done:
  spmv_drop(c, pf);
  user_wave_done(c, li);
}

// Roofline probe: waves copy 4 KiB blocks from `src` (pinned host or HBM) to `dst`
// (HBM), `per` blocks in flight per wave, with the same wave-cooperative copy the emulated
// controller uses.  Block i is src block `list[i]` (or i when list is NULL) and lands in
// dst block (i % dst_blocks).
__global__ __launch_bounds__(WG) void k_probe_copy(const uint8_t* src, const uint64_t* list, uint64_t n,
                                                   uint8_t* dst, uint64_t dst_blocks, uint32_t per) {
  const uint32_t w = blockIdx.x * WPB + threadIdx.x / 64;
  const uint32_t W = gridDim.x * WPB;
  for (uint64_t i0 = (uint64_t)w * per; i0 < n; i0 += (uint64_t)W * per) {
    uint8_t* d[4];
    const uint8_t* s[4];
    uint32_t k = 0;
    for (uint32_t j = 0; j < per && i0 + j < n; ++j) {
      const uint64_t i = i0 + j;
      const uint64_t b = list ? list[i] : i;
      s[k] = src + (b << 12);
      d[k] = dst + ((i % dst_blocks) << 12);
      ++k;
    }
    copy_blocks(d, s, k);
  }
}

// Debug dump: tag (or -1), state, pin count per line.
__global__ void k_dump(dev_ctx c, int64_t* tags, uint8_t* states, uint32_t* rc) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < c.num_lines) {
    const uint64_t m = ld_rlx(c.meta + i);
    tags[i] = m_state(m) == ST_INVALID ? -1 : (int64_t)m_tag(m);
    states[i] = (uint8_t)m_state(m);
    rc[i] = m_rc(m);
  }
}

}  // namespace

// =============================================================================== host side
static constexpr size_t bwd_al(size_t v) { return (v + 255) & ~(size_t)255; }

// Work area of a backward launch over n lookups: sort keys, the bag of every lookup
// position, the heads of the distinct rows, two counters and the radix sort's own area.
static constexpr size_t bwd_work_bytes(uint64_t n) {
  return bwd_al(n * 8) + bwd_al(n * 4) + bwd_al(n * 4) + 256 + sort::radix_work_bytes(n);
}

// Work area of the allocation-free backward entry point: one fixed array per device,
// shared by every call on that device (see agile_embbag_backward_sgd_noalloc), about
// 25 MiB for up to 2^20 lookups per call.  In host code `scratch` only names the symbol;
// its device address comes from hipGetSymbolAddress, taken once per device at
// agile_init and kept in scratch_dev.
constexpr uint64_t NOALLOC_MAX_LOOKUPS = 1ull << 20;
constexpr size_t NOALLOC_SCRATCH_BYTES = bwd_work_bytes(NOALLOC_MAX_LOOKUPS);
static __device__ __align__(256) uint8_t scratch[NOALLOC_SCRATCH_BYTES];
constexpr int MAX_DEVICES = 64;
static void* scratch_dev[MAX_DEVICES];
static std::mutex scratch_mu;

struct agile_store_s {
  void* host[AGILE_MAX_DEVICES];
  uint8_t* dev[AGILE_MAX_DEVICES];  // device addresses of the pinned images
  uint32_t n_dev;
  uint64_t bytes;       // logical store
  uint64_t blocks;
  uint64_t dev_bytes;   // per device
};

struct session_req {
  uint64_t id, bag0, nb, look0, nl, lines;
  bool polled;
};
// Largest request a session accepts (lookups, and bags).
constexpr uint64_t SESSION_MAX_LOOKUPS = 1ull << 16;

struct agile_session_s {
  agile_ctx ctx = nullptr;
  agile_tables tb{};
  uint64_t bag_cap = 0, look_cap = 0, req_cap = 0;  // ring sizes (powers of two)
  uint64_t cap_look = 0, cap_lines = 0, cap_req = 0;  // admission budgets
  void* host = nullptr;  // pinned, mapped, coherent: control words and rings
  void* dev = nullptr;   // HBM: per-request-slot bag counters, staged count, ring copies
  hipStream_t hs = nullptr;
  uint64_t* ctl = nullptr;  // [0] bags published, [1] stop
  uint64_t *bag_j0 = nullptr, *bag_j1 = nullptr, *bag_req = nullptr;
  uint32_t* bag_tab = nullptr;
  int64_t* idx = nullptr;
  uint32_t *req_nbags = nullptr, *done = nullptr;
  float* out = nullptr;
  uint64_t next_req = 0, next_bag = 0, next_look = 0;
  uint64_t in_look = 0, in_lines = 0;
  uint64_t user_waves = 0;
  std::deque<session_req> live;  // submitted and not yet collected, in submission order
};

struct agile_ctx_s {
  agile_config cfg;
  agile_session_s* session = nullptr;  // an open serving session owns the device
  dev_ctx d;
  uint32_t n_ctrl, n_cq, service_blocks;
  uint32_t cu_count;
  uint64_t clock_hz;
  agile_store_s* store = nullptr;
  std::string last_error;
  bool poisoned = false;
  uint32_t* abort_host = nullptr;  // pinned, mapped
  std::vector<void*> dev_allocs;
  std::vector<int> occ_cache;  // resident workgroups per CU, per kernel kind
  void* scratch = nullptr;     // backward-pass work arrays, grown on demand
  size_t scratch_bytes = 0;
  uint32_t iso_lds = 0;        // LDS per workgroup that makes one workgroup fill a CU
  std::vector<std::pair<const void*, uint32_t>> dyn_lds;  // per kernel: dynamic LDS to add
  void* noalloc_scratch = nullptr;  // device address of `scratch` on this context's device
  uint32_t* defer_list = nullptr;   // bags the resident-hit pass leaves to the I/O pass
  uint64_t defer_cap = 0;
};

namespace {

constexpr int KIND_EMBBAG1 = 0, KIND_EMBBAG2 = 1, KIND_EMBBAG4 = 2, KIND_READ = 3, KIND_FLUSH = 4,
              KIND_TRACE = 5, KIND_BWD1 = 6, KIND_BWD2 = 7, KIND_BWD4 = 8, KIND_SERVE1 = 9,
              KIND_SERVE2 = 10, KIND_SERVE4 = 11, KIND_WRITE = 12, KIND_ISSUE = 13, KIND_WBACK = 14,
              KIND_PF1 = 15, KIND_PF2 = 16, KIND_PF4 = 17, KIND_N = 18;

agile_status fail(agile_ctx ctx, agile_status s, const std::string& msg) {
  if (ctx) ctx->last_error = msg;
  return s;
}

#define HIPCHK(ctx, call)                                                                   \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess) {                                                                 \
      return fail(ctx, AGILE_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));       \
    }                                                                                       \
  } while (0)

bool is_pow2(uint64_t v) { return v && !(v & (v - 1)); }
uint32_t log2u(uint64_t v) {
  uint32_t r = 0;
  while ((1ull << r) < v) ++r;
  return r;
}

template <class T>
agile_status dalloc(agile_ctx ctx, T** p, size_t bytes) {
  void* q = nullptr;
  if (hipMalloc(&q, bytes ? bytes : 64) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, AGILE_ENOMEM, "hipMalloc failed for " + std::to_string(bytes) + " bytes");
  }
  ctx->dev_allocs.push_back(q);
  *p = reinterpret_cast<T*>(q);
  return AGILE_OK;
}

// Dynamic LDS a launch of kernel f adds (see agile_init).
uint32_t lds_of(agile_ctx ctx, const void* f) {
  for (const auto& e : ctx->dyn_lds)
    if (e.first == f) return e.second;
  return 0;
}

int occupancy(agile_ctx ctx, int kind) {
  int& v = ctx->occ_cache[kind];
  if (v > 0) return v;
  int nb = 0;
  hipError_t e = hipSuccess;
  const void* f;
  switch (kind) {
    case KIND_EMBBAG1: f = (const void*)k_embbag<1>; break;
    case KIND_EMBBAG2: f = (const void*)k_embbag<2>; break;
    case KIND_EMBBAG4: f = (const void*)k_embbag<4>; break;
    case KIND_READ: f = (const void*)k_async_read; break;
    case KIND_FLUSH: f = (const void*)k_flush; break;
    case KIND_WRITE: f = (const void*)k_write_lines; break;
    case KIND_ISSUE: f = (const void*)k_async_issue; break;
    case KIND_WBACK: f = (const void*)k_buf_writeback; break;
    case KIND_BWD1: f = (const void*)k_bwd_sgd<1>; break;
    case KIND_BWD2: f = (const void*)k_bwd_sgd<2>; break;
    case KIND_BWD4: f = (const void*)k_bwd_sgd<4>; break;
    case KIND_SERVE1: f = (const void*)k_serve<1>; break;
    case KIND_SERVE2: f = (const void*)k_serve<2>; break;
    case KIND_SERVE4: f = (const void*)k_serve<4>; break;
    case KIND_PF1: f = (const void*)k_embbag_pf<1>; break;
    case KIND_PF2: f = (const void*)k_embbag_pf<2>; break;
    case KIND_PF4: f = (const void*)k_embbag_pf<4>; break;
    default: f = (const void*)k_trace; break;
  }
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, WG, lds_of(ctx, f));
  if (e != hipSuccess || nb <= 0) nb = 1;
  v = nb;
  return v;
}

// User wavefronts a launch of `kind` may use so that the whole grid (service included)
// is resident at once.
uint32_t user_wave_cap(agile_ctx ctx, int kind, uint32_t service_blocks) {
  const uint64_t blocks = (uint64_t)occupancy(ctx, kind) * ctx->cu_count;
  uint64_t ub = blocks > service_blocks ? blocks - service_blocks : 1;
  uint64_t uw = ub * WPB;
  if (ctx->cfg.max_user_waves && uw > ctx->cfg.max_user_waves) uw = ctx->cfg.max_user_waves;
  return (uint32_t)std::max<uint64_t>(uw, 1);
}
uint32_t user_wave_cap(agile_ctx ctx, int kind) { return user_wave_cap(ctx, kind, ctx->service_blocks); }

agile_status check_usable(agile_ctx ctx) {
  if (!ctx) return AGILE_EINVAL;
  if (ctx->poisoned) return fail(ctx, AGILE_ESTATE, "context has a sticky device error");
  if (ctx->session) return fail(ctx, AGILE_ESTATE, "a serving session is open on this context");
  return AGILE_OK;
}

// user_waves must be a multiple of WPB (every wave of a user workgroup reports done).
// The launch descriptor holds no host-side running totals: a captured launch replays.
launch_t make_launch(agile_ctx ctx, uint32_t user_waves, bool service) {
  launch_t li{};
  li.service_blocks = service ? ctx->service_blocks : 0;
  li.n_ctrl = ctx->n_ctrl;
  li.n_cq = ctx->n_cq;
  li.user_waves = user_waves;
  li.prio = (ctx->cfg.flags & AGILE_F_NO_PRIO) ? 0 : 1;
  return li;
}

agile_status bind_store(agile_ctx ctx) {
  if (ctx->store) {
    const agile_store_s* st = ctx->store;
    uint64_t tab[AGILE_MAX_DEVICES] = {};
    for (uint32_t d = 0; d < st->n_dev; ++d) tab[d] = (uint64_t)(uintptr_t)st->dev[d];
    HIPCHK(ctx, hipMemcpy((void*)ctx->d.dev_image, tab, sizeof(tab), hipMemcpyHostToDevice));
    ctx->d.image = st->dev[0];
    ctx->d.store_blocks = st->blocks;
    ctx->d.dev_blocks = st->dev_bytes / 4096;
    ctx->d.n_dev = st->n_dev;
  } else {
    ctx->d.image = nullptr;
    ctx->d.store_blocks = 0;
    ctx->d.dev_blocks = 0;
    ctx->d.n_dev = 1;
  }
  return AGILE_OK;
}

// Text of a recorded lock chain (see lc_walk); empty when none was recorded.
static std::string wait_text(uint64_t what, uint64_t word) {
  const uint32_t kind = (uint32_t)(what >> 56);
  const unsigned long long id = what & ((1ull << 56) - 1);
  char b[200];
  switch (kind) {
    case W_SQ_SLOT:
      snprintf(b, sizeof b, "a free slot of SQ %llu for ticket %llu (slot word 0x%llx)", id >> 32, id & 0xFFFFFFFFull,
               (unsigned long long)word);
      break;
    case W_SETLOCK:
      if (word >= 2)
        snprintf(b, sizeof b, "the set lock of store line %llu, held by wave %llu", id, (unsigned long long)word - 2);
      else
        snprintf(b, sizeof b, "the set lock of store line %llu (%s)", id, word ? "held" : "free now");
      break;
    case W_WB:
    case W_FILL:
    case W_TICKET:
    case W_CLAIM:
      snprintf(b, sizeof b, "%s of cache line %llu (state %llu, pins %llu, tag %llu)",
               kind == W_WB ? "its write-back" : (kind == W_FILL ? "the fill" : (kind == W_TICKET ? "the ticket's line" : "a write claim")),
               id, (unsigned long long)(word & 7), (unsigned long long)((word >> 4) & 0xFFFFF), (unsigned long long)(word >> 32));
      break;
    case W_WAY: snprintf(b, sizeof b, "an evictable way (after EAGAIN, object %llu)", id); break;
    case W_BACKLOG: snprintf(b, sizeof b, "fewer than %llu commands in flight (prefetch)", id); break;
    case 0: snprintf(b, sizeof b, "nothing (running)"); break;
    default: snprintf(b, sizeof b, "0x%llx", (unsigned long long)what); break;
  }
  return b;
}
static std::string format_chain(const uint64_t* ch) {
  if (!(ch[0] >> 63)) return "";
  const uint32_t n = (uint32_t)((ch[0] >> 1) & 0xFFFF);
  const bool cycle = ch[0] & 1;
  std::string t = "; lock chain:";
  for (uint32_t i = 0; i < n && i < LC_MAX; ++i) {
    t += (i ? "; " : " ") + std::string("wave ") + std::to_string(ch[1 + 3 * i]) + " waits for " +
         wait_text(ch[2 + 3 * i], ch[3 + 3 * i]);
  }
  if (cycle) t += "; a cycle back to wave " + std::to_string(ch[1 + 3 * n]);
  return t;
}

agile_status map_device_error(agile_ctx ctx) {
  uint32_t err = 0;
  uint64_t info = 0;
  HIPCHK(ctx, hipMemcpy(&err, ctx->d.err, sizeof(err), hipMemcpyDeviceToHost));
  HIPCHK(ctx, hipMemcpy(&info, ctx->d.err_info, sizeof(info), hipMemcpyDeviceToHost));
  if (!err && !*ctx->abort_host) return AGILE_OK;
  ctx->poisoned = true;
  char buf[160];
  snprintf(buf, sizeof buf, "device error %u (info 0x%llx)", err, (unsigned long long)info);
  std::string chain;
  if (ctx->cfg.flags & AGILE_F_LOCKCHAIN) {
    std::vector<uint64_t> ch(1 + 3 * LC_MAX + 1, 0);
    if (hipMemcpy(ch.data(), ctx->d.chain, ch.size() * 8, hipMemcpyDeviceToHost) == hipSuccess)
      chain = format_chain(ch.data());
  }
  switch (err) {
    case E_TIMEDOUT: return fail(ctx, AGILE_ETIMEDOUT, std::string(buf) + ": watchdog timeout" + chain);
    case E_IO: return fail(ctx, AGILE_EIO, std::string(buf) + ": command error status");
    case E_PROTO: return fail(ctx, AGILE_EPROTO, std::string(buf) + ": queue protocol violation");
    case E_STATE: return fail(ctx, AGILE_ESTATE, std::string(buf) + ": invalid state or argument");
    default: return fail(ctx, AGILE_ETIMEDOUT, std::string(buf) + ": aborted");
  }
}

// Host-side watchdog: polls the stream; past the limit it raises the pinned abort flag
// (every device wait checks it) and keeps waiting for the kernels to drain.
agile_status sync_stream(agile_ctx ctx, hipStream_t s) {
  const double limit_s = 4.0 * (double)ctx->cfg.timeout_ns * 1e-9 + 30.0;
  auto t0 = std::chrono::steady_clock::now();
  bool raised = false;
  for (;;) {
    hipError_t e = hipStreamQuery(s);
    if (e == hipSuccess) break;
    if (e != hipErrorNotReady) return fail(ctx, AGILE_EHIP, std::string("hipStreamQuery: ") + hipGetErrorString(e));
    const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (!raised && el > limit_s) {
      __atomic_store_n(ctx->abort_host, 1u, __ATOMIC_SEQ_CST);
      raised = true;
    }
    if (raised && el > 2 * limit_s) {
      ctx->poisoned = true;
      return fail(ctx, AGILE_ETIMEDOUT, "stream did not drain after the abort flag was raised");
    }
    std::this_thread::sleep_for(std::chrono::microseconds(el < 0.01 ? 20 : 500));
  }
  return map_device_error(ctx);
}

}  // namespace

// ------------------------------------------------------------------------ public API
extern "C" {

const char* agile_status_string(agile_status s) {
  switch (s) {
    case AGILE_OK: return "AGILE_OK";
    case AGILE_EINVAL: return "AGILE_EINVAL: invalid argument or configuration";
    case AGILE_ENOMEM: return "AGILE_ENOMEM: allocation failed";
    case AGILE_EHIP: return "AGILE_EHIP: HIP runtime error";
    case AGILE_ETIMEDOUT: return "AGILE_ETIMEDOUT: device watchdog timeout";
    case AGILE_EAGAIN: return "AGILE_EAGAIN: no evictable line; retry";
    case AGILE_EIO: return "AGILE_EIO: command completed with error status";
    case AGILE_EPROTO: return "AGILE_EPROTO: queue protocol violation";
    case AGILE_ESTATE: return "AGILE_ESTATE: call not allowed in this state";
  }
  return "unknown agile_status";
}

const char* agile_last_error(agile_ctx ctx) {
  return ctx ? ctx->last_error.c_str() : "no context";
}

void agile_config_default(agile_config* cfg) {
  if (!cfg) return;
  memset(cfg, 0, sizeof(*cfg));
  cfg->struct_size = sizeof(agile_config);
  cfg->device = 0;
  cfg->cache_bytes = 1ull << 20;
  cfg->line_bytes = 4096;
  cfg->assoc = 8;
  cfg->num_qp = 1;
  cfg->qp_depth = 64;
  cfg->timeout_ns = 10ull * 1000000000ull;
}

agile_status agile_init(const agile_config* cfg_in, agile_ctx* out) {
  if (!cfg_in || !out) return AGILE_EINVAL;
  *out = nullptr;
  if (cfg_in->struct_size != sizeof(agile_config)) return AGILE_EINVAL;
  agile_config cfg = *cfg_in;
  if (cfg.timeout_ns == 0) cfg.timeout_ns = 10ull * 1000000000ull;
  // ---- validation (no device work before this point)
  if (cfg.line_bytes < 4096 || !is_pow2(cfg.line_bytes) || cfg.line_bytes > (1u << 26)) return AGILE_EINVAL;
  if (cfg.cache_bytes == 0 || cfg.cache_bytes % cfg.line_bytes) return AGILE_EINVAL;
  const uint64_t lines = cfg.cache_bytes / cfg.line_bytes;
  if (cfg.assoc == 0 || lines < cfg.assoc || lines % cfg.assoc) return AGILE_EINVAL;
  if (lines > 0xFFFFFFFFull) return AGILE_EINVAL;
  if (cfg.num_qp == 0 || cfg.num_qp > 1024) return AGILE_EINVAL;
  if (cfg.qp_depth < 64 || cfg.qp_depth > 65536 || !is_pow2(cfg.qp_depth)) return AGILE_EINVAL;
  // by default enough controller wavefronts that their PCIe copies are not the limit
  uint32_t n_ctrl = cfg.ctrl_waves ? cfg.ctrl_waves : std::max<uint32_t>(cfg.num_qp, 64);
  uint32_t n_cq = cfg.cq_waves ? cfg.cq_waves : std::min<uint32_t>(cfg.num_qp, 64);
  if (n_ctrl > 4096 || n_cq > 1024) return AGILE_EINVAL;
  if ((uint64_t)n_cq * 64 < cfg.num_qp) return AGILE_EINVAL;  // <= 64 CQs per polling wave
  if (n_cq > cfg.num_qp) n_cq = cfg.num_qp;

  agile_ctx ctx = new agile_ctx_s();
  ctx->cfg = cfg;
  ctx->occ_cache.assign(KIND_N, 0);
  auto bail = [&](agile_status s) {
    agile_shutdown(ctx);
    return s;
  };
  if (hipSetDevice(cfg.device) != hipSuccess) {
    (void)hipGetLastError();
    delete ctx;
    return AGILE_EHIP;
  }
  if (cfg.device < 0 || cfg.device >= MAX_DEVICES) {
    delete ctx;
    return AGILE_EINVAL;
  }
  {
    // the allocation-free entry point's work area on this device (the current one)
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (!scratch_dev[cfg.device]) {
      void* p = nullptr;
      if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
        (void)hipGetLastError();
        delete ctx;
        return AGILE_EHIP;
      }
      scratch_dev[cfg.device] = p;
    }
    ctx->noalloc_scratch = scratch_dev[cfg.device];
  }
  int cus = 0, wclk_khz = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, cfg.device) != hipSuccess ||
      hipDeviceGetAttribute(&wclk_khz, hipDeviceAttributeWallClockRate, cfg.device) != hipSuccess) {
    delete ctx;
    return AGILE_EHIP;
  }
  ctx->cu_count = (uint32_t)cus;
  ctx->clock_hz = (uint64_t)wclk_khz * 1000ull;
  {
    // more than half a CU's LDS per workgroup: one workgroup per CU for service kernels
    int lds_cu = 0;
    if (hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, cfg.device) != hipSuccess)
      lds_cu = 0;
    // (a kernel whose own static LDS is already that large adds nothing)
    const uint32_t iso = lds_cu > 0 ? (uint32_t)((lds_cu / 2 + 1024 + 255) & ~255) : 0u;
    const void* fns[] = {(const void*)k_async_read, (const void*)k_flush, (const void*)k_embbag<1>,
                         (const void*)k_embbag<2>, (const void*)k_embbag<4>, (const void*)k_bfs_front,
                         (const void*)k_bfs_edges, (const void*)k_spmv, (const void*)k_bwd_sgd<1>,
                         (const void*)k_bwd_sgd<2>, (const void*)k_bwd_sgd<4>, (const void*)k_serve<1>,
                         (const void*)k_serve<2>, (const void*)k_serve<4>, (const void*)k_trace,
                         (const void*)k_write_lines, (const void*)k_async_issue, (const void*)k_buf_writeback,
                         (const void*)k_embbag_pf<1>, (const void*)k_embbag_pf<2>, (const void*)k_embbag_pf<4>};
    for (const void* f : fns) {
      hipFuncAttributes fa;
      memset(&fa, 0, sizeof(fa));
      uint32_t dyn = 0;
      if (iso && hipFuncGetAttributes(&fa, f) == hipSuccess) {
        const uint32_t st = (uint32_t)fa.sharedSizeBytes;
        dyn = st < iso ? iso - st : 0u;
        if (dyn && hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn) != hipSuccess) dyn = 0;
      }
      (void)hipGetLastError();
      ctx->dyn_lds.emplace_back(f, dyn);
    }
    ctx->iso_lds = iso;
  }
  ctx->n_ctrl = n_ctrl;
  ctx->n_cq = n_cq;
  ctx->service_blocks = service_blocks_for(n_ctrl + n_cq);

  dev_ctx& d = ctx->d;
  memset(&d, 0, sizeof(d));
  d.num_lines = (uint32_t)lines;
  d.assoc = cfg.assoc;
  d.num_sets = (uint32_t)(lines / cfg.assoc);
  d.sets_pow2 = is_pow2(d.num_sets) ? 1u : 0u;
  d.line_shift = log2u(cfg.line_bytes);
  d.blocks_per_line = cfg.line_bytes / 4096;
  d.num_qp = cfg.num_qp;
  d.depth = cfg.qp_depth;
  d.depth_shift = log2u(cfg.qp_depth);
  d.lat_ticks = (uint64_t)((double)cfg.latency_ns * 1e-9 * (double)ctx->clock_hz + 0.5);
  d.tok_fp = cfg.iops_cap ? (uint64_t)((double)ctx->clock_hz / (double)cfg.iops_cap * (double)(1ull << TOK_FRAC)) : 0;
  {
    // every command that can be queued or held by a controller lane, one period each
    const double lim = ((double)cfg.num_qp * cfg.qp_depth + 64.0 * n_ctrl) * (double)d.tok_fp;
    d.tok_max = lim < 4.0e18 ? (uint64_t)lim : 4000000000000000000ull;
  }
  d.timeout_ticks = (uint64_t)((double)cfg.timeout_ns * 1e-9 * (double)ctx->clock_hz);
  d.flags = cfg.flags;

  agile_status s;
  const uint64_t nq = (uint64_t)cfg.num_qp * cfg.qp_depth;
  if ((s = dalloc(ctx, &d.lines, cfg.cache_bytes)) != AGILE_OK) return bail(s);
  if ((s = dalloc(ctx, &d.meta, lines * 8)) != AGILE_OK) return bail(s);
  if ((s = dalloc(ctx, &d.hand, (uint64_t)d.num_sets * 4)) != AGILE_OK) return bail(s);
  if ((s = dalloc(ctx, &d.set_lock, (uint64_t)d.num_sets * 4)) != AGILE_OK) return bail(s);
  if ((s = dalloc(ctx, &d.sq, nq * sizeof(sqe_t))) != AGILE_OK) return bail(s);
  if ((s = dalloc(ctx, &d.cq, nq * sizeof(cqe_t))) != AGILE_OK) return bail(s);
  if ((s = dalloc(ctx, &d.slot, nq * 4)) != AGILE_OK) return bail(s);
  if ((s = dalloc(ctx, &d.qp, (uint64_t)cfg.num_qp * sizeof(qp_t))) != AGILE_OK) return bail(s);
  if ((s = dalloc(ctx, &d.next_tok, 128 * AGILE_MAX_DEVICES)) != AGILE_OK) return bail(s);
  uint64_t* dev_tab = nullptr;
  if ((s = dalloc(ctx, &dev_tab, 8 * AGILE_MAX_DEVICES)) != AGILE_OK) return bail(s);
  d.dev_image = dev_tab;
  d.n_dev = 1;
  if ((s = dalloc(ctx, &d.cnt, (uint64_t)C_COUNT * CSTRIDE * 8)) != AGILE_OK) return bail(s);
  ctx->defer_cap = 1ull << 20;  // bags per launch the resident-hit pass can take (4 MiB list)
  if ((s = dalloc(ctx, &ctx->defer_list, ctx->defer_cap * 4)) != AGILE_OK) return bail(s);
  if ((s = dalloc(ctx, &d.err, 128)) != AGILE_OK) return bail(s);
  if ((s = dalloc(ctx, &d.waits, 16ull * WAIT_SLOTS)) != AGILE_OK) return bail(s);
  if ((s = dalloc(ctx, &d.chain, 8ull * (1 + 3 * LC_MAX) + 8)) != AGILE_OK) return bail(s);
  if ((s = dalloc(ctx, &d.pend_head, 4ull * lines)) != AGILE_OK) return bail(s);
  if ((s = dalloc(ctx, &d.pend, 16ull * PEND_CAP)) != AGILE_OK) return bail(s);
  if ((s = dalloc(ctx, &d.share_key, 8ull * SHARE_CAP)) != AGILE_OK) return bail(s);
  if ((s = dalloc(ctx, &d.share_buf, 8ull * SHARE_CAP)) != AGILE_OK) return bail(s);
  if ((s = dalloc(ctx, &d.share_refs, 4ull * SHARE_CAP)) != AGILE_OK) return bail(s);
  if ((s = dalloc(ctx, &d.err_info, 128)) != AGILE_OK) return bail(s);
  if ((s = dalloc(ctx, &d.abort_dev, 128)) != AGILE_OK) return bail(s);
  void* ab = nullptr;
  if (hipHostMalloc(&ab, 4096, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
    (void)hipGetLastError();
    return bail(AGILE_ENOMEM);
  }
  ctx->abort_host = (uint32_t*)ab;
  *ctx->abort_host = 0;
  void* abd = nullptr;
  if (hipHostGetDevicePointer(&abd, ab, 0) != hipSuccess) return bail(AGILE_EHIP);
  d.abort_flag = (uint32_t*)abd;

  // zero state; SQ slot s starts as EMPTY for ticket s
  if (hipMemset(d.meta, 0, lines * 8) != hipSuccess || hipMemset(d.hand, 0, (uint64_t)d.num_sets * 4) != hipSuccess ||
      hipMemset(d.set_lock, 0, (uint64_t)d.num_sets * 4) != hipSuccess ||
      hipMemset(d.sq, 0, nq * sizeof(sqe_t)) != hipSuccess || hipMemset(d.cq, 0, nq * sizeof(cqe_t)) != hipSuccess ||
      hipMemset(d.qp, 0, (uint64_t)cfg.num_qp * sizeof(qp_t)) != hipSuccess || hipMemset(d.next_tok, 0, 128 * AGILE_MAX_DEVICES) != hipSuccess ||
      hipMemset(d.cnt, 0, (uint64_t)C_COUNT * CSTRIDE * 8) != hipSuccess || hipMemset(d.err, 0, 128) != hipSuccess ||
      hipMemset(d.err_info, 0, 128) != hipSuccess || hipMemset(d.abort_dev, 0, 128) != hipSuccess ||
      hipMemset(d.waits, 0, 16ull * WAIT_SLOTS) != hipSuccess ||
      hipMemset(d.chain, 0, 8ull * (1 + 3 * LC_MAX) + 8) != hipSuccess ||
      hipMemset(d.pend_head, 0xFF, 4ull * lines) != hipSuccess ||  // PEND_EMPTY
      hipMemset(d.share_key, 0, 8ull * SHARE_CAP) != hipSuccess ||
      hipMemset(d.share_refs, 0, 4ull * SHARE_CAP) != hipSuccess)
    return bail(AGILE_EHIP);
  std::vector<uint32_t> slots(nq);
  for (uint64_t i = 0; i < nq; ++i) slots[i] = (uint32_t)((i % cfg.qp_depth) << 2) | SLOT_EMPTY;
  if (hipMemcpy(d.slot, slots.data(), nq * 4, hipMemcpyHostToDevice) != hipSuccess) return bail(AGILE_EHIP);
  if (hipDeviceSynchronize() != hipSuccess) return bail(AGILE_EHIP);
  *out = ctx;
  return AGILE_OK;
}

agile_status agile_shutdown(agile_ctx ctx) {
  if (!ctx) return AGILE_EINVAL;
  if (ctx->session) (void)agile_session_close(ctx->session);
  (void)hipDeviceSynchronize();
  for (void* p : ctx->dev_allocs) (void)hipFree(p);
  if (ctx->abort_host) (void)hipHostFree(ctx->abort_host);
  if (ctx->scratch) (void)hipFree(ctx->scratch);
  delete ctx->store;
  delete ctx;
  return AGILE_OK;
}

agile_status agile_host_alloc(uint64_t bytes, void** out) {
  if (!out || bytes == 0) return AGILE_EINVAL;
  *out = nullptr;
  // Non-coherent pinned memory: the GPU reads it through its L2 in whole cache lines
  // (one PCIe request per line instead of one per 16-byte lane access).  The emulated
  // controller invalidates with system scope before every copy batch and releases with
  // system scope after writing, so both directions stay correct.
  if (hipHostMalloc(out, bytes, hipHostMallocMapped | hipHostMallocNonCoherent) != hipSuccess) {
    (void)hipGetLastError();
    return AGILE_ENOMEM;
  }
  return AGILE_OK;
}

agile_status agile_host_free(void* p) {
  if (!p) return AGILE_EINVAL;
  return hipHostFree(p) == hipSuccess ? AGILE_OK : AGILE_EHIP;
}

agile_status agile_open_store(agile_ctx ctx, void* host_image, uint64_t bytes, uint32_t block_bytes,
                              uint32_t flags, agile_store* out) {
  void* const images[1] = {host_image};
  return agile_open_store_striped(ctx, images, 1, bytes, block_bytes, flags, out);
}

agile_status agile_open_store_striped(agile_ctx ctx, void* const* host_images, uint32_t n, uint64_t bytes_each,
                                      uint32_t block_bytes, uint32_t flags, agile_store* out) {
  agile_status s = check_usable(ctx);
  if (s) return s;
  if (!host_images || !out || block_bytes != 4096 || bytes_each == 0 || bytes_each % block_bytes)
    return fail(ctx, AGILE_EINVAL, "open_store: images must be non-null, block_bytes 4096, bytes a multiple of it");
  if (n == 0 || n > AGILE_MAX_DEVICES) return fail(ctx, AGILE_EINVAL, "open_store: 1..AGILE_MAX_DEVICES devices");
  (void)flags;
  if (ctx->store) return fail(ctx, AGILE_ESTATE, "open_store: a store is already open on this context");
  const uint64_t line_bytes = 1ull << ctx->d.line_shift;
  if (n > 1 && (bytes_each % line_bytes || ctx->d.num_qp % n))
    return fail(ctx, AGILE_EINVAL,
                "open_store: with several devices each holds whole lines and the queue pairs divide evenly");
  const uint64_t bytes = bytes_each * n;
  if ((bytes / 4096 + ctx->d.blocks_per_line - 1) / ctx->d.blocks_per_line >= 0xFFFFFFFFull)
    return fail(ctx, AGILE_EINVAL, "open_store: store too large for 32-bit line ids");
  agile_store st = new agile_store_s();
  for (uint32_t d = 0; d < n; ++d) {
    hipPointerAttribute_t attr;
    memset(&attr, 0, sizeof(attr));
    if (!host_images[d] || hipPointerGetAttributes(&attr, host_images[d]) != hipSuccess ||
        attr.type != hipMemoryTypeHost || attr.devicePointer == nullptr) {
      (void)hipGetLastError();
      delete st;
      return fail(ctx, AGILE_EINVAL, "open_store: an image is not pinned, device-mapped host memory");
    }
    st->host[d] = host_images[d];
    st->dev[d] = (uint8_t*)attr.devicePointer + ((uint8_t*)host_images[d] - (uint8_t*)attr.hostPointer);
  }
  st->n_dev = n;
  st->bytes = bytes;
  st->blocks = bytes / 4096;
  st->dev_bytes = bytes_each;
  ctx->store = st;
  if ((s = bind_store(ctx)) != AGILE_OK) {
    ctx->store = nullptr;
    delete st;
    (void)bind_store(ctx);
    return s;
  }
  *out = st;
  return AGILE_OK;
}

agile_status agile_write(agile_ctx ctx, agile_store store, const uint64_t* d_lines, uint32_t n, const void* d_src,
                         void* stream) {
  agile_status s = check_usable(ctx);
  if (s) return s;
  if (store != ctx->store) return fail(ctx, AGILE_EINVAL, "write: store is not open on this context");
  if (n == 0) return AGILE_OK;
  if (!d_lines || !d_src) return fail(ctx, AGILE_EINVAL, "write: null pointer");
  if (store->bytes % (1ull << ctx->d.line_shift))
    return fail(ctx, AGILE_EINVAL, "write: the store must hold whole lines");
  hipStream_t hs = (hipStream_t)stream;
  // a wave pins at most one chunk (64 lines) at a time
  const uint64_t by_cache = std::max<uint64_t>(1, ctx->d.num_lines / 64);
  uint32_t uw = (uint32_t)std::min<uint64_t>({(n + 63) / 64, (uint64_t)user_wave_cap(ctx, KIND_WRITE), by_cache});
  uw = (uw + WPB - 1) / WPB * WPB;
  launch_t li = make_launch(ctx, uw, true);
  hipLaunchKernelGGL(k_write_lines, dim3(li.service_blocks + uw / WPB), dim3(WG),
                     lds_of(ctx, (const void*)k_write_lines), hs, ctx->d, li, d_lines, n, (const uint8_t*)d_src);
  HIPCHK(ctx, hipGetLastError());
  return sync_stream(ctx, hs);
}

agile_status agile_sync(agile_ctx ctx, void* stream) {
  if (!ctx) return AGILE_EINVAL;
  return sync_stream(ctx, (hipStream_t)stream);
}

agile_status agile_invalidate(agile_ctx ctx, agile_store store, void* stream) {
  agile_status s = check_usable(ctx);
  if (s) return s;
  if (store != ctx->store) return fail(ctx, AGILE_EINVAL, "invalidate: store is not open on this context");
  hipStream_t hs = (hipStream_t)stream;
  uint64_t waves = std::max<uint64_t>((std::max<uint64_t>(ctx->d.num_lines, ctx->d.num_sets) + 63) / 64, 1);
  waves = (waves + WPB - 1) / WPB * WPB;
  launch_t li = make_launch(ctx, (uint32_t)waves, false);
  hipLaunchKernelGGL(k_invalidate, dim3((uint32_t)(waves / WPB)), dim3(WG), 0, hs, ctx->d, li);
  HIPCHK(ctx, hipGetLastError());
  return sync_stream(ctx, hs);
}

agile_status agile_close_store(agile_ctx ctx, agile_store store) {
  if (!ctx || !store || store != ctx->store) return fail(ctx, AGILE_EINVAL, "close_store: unknown store");
  if (ctx->session) return fail(ctx, AGILE_ESTATE, "close_store: a serving session is open");
  agile_status s = AGILE_OK;
  if (!ctx->poisoned) {
    s = sync_stream(ctx, nullptr);
    if (s == AGILE_OK) {
      HIPCHK(ctx, hipDeviceSynchronize());
      // drop clean lines; dirty lines are discarded too (documented: flush first)
      HIPCHK(ctx, hipMemset(ctx->d.meta, 0, (uint64_t)ctx->d.num_lines * 8));
      HIPCHK(ctx, hipMemset(ctx->d.hand, 0, (uint64_t)ctx->d.num_sets * 4));
      HIPCHK(ctx, hipDeviceSynchronize());
    }
  }
  ctx->store = nullptr;
  bind_store(ctx);
  delete store;
  return s;
}

agile_status agile_async_read(agile_ctx ctx, agile_store store, const uint64_t* d_blocks, uint32_t n,
                              agile_ticket* d_tickets, void* stream) {
  agile_status s = check_usable(ctx);
  if (s) return s;
  if (store != ctx->store) return fail(ctx, AGILE_EINVAL, "async_read: store is not open on this context");
  if (n == 0) return AGILE_OK;
  if (!d_blocks || !d_tickets) return fail(ctx, AGILE_EINVAL, "async_read: null pointer");
  uint32_t uw = std::min<uint32_t>((n + 63) / 64, user_wave_cap(ctx, KIND_READ));
  uw = (uw + WPB - 1) / WPB * WPB;
  launch_t li = make_launch(ctx, uw, true);
  hipLaunchKernelGGL(k_async_read, dim3(li.service_blocks + uw / WPB), dim3(WG), lds_of(ctx, (const void*)k_async_read), (hipStream_t)stream,
                     ctx->d, li, d_blocks, n, d_tickets);
  HIPCHK(ctx, hipGetLastError());
  return AGILE_OK;
}

agile_status agile_wait(agile_ctx ctx, const agile_ticket* d_tickets, uint32_t n, void** d_ptrs, void* stream) {
  agile_status s = check_usable(ctx);
  if (s) return s;
  if (n && (!d_tickets || !d_ptrs)) return fail(ctx, AGILE_EINVAL, "wait: null pointer");
  hipStream_t hs = (hipStream_t)stream;
  uint64_t e0 = 0;
  HIPCHK(ctx, hipMemcpy(&e0, ctx->d.cnt + (size_t)C_AUX0 * CSTRIDE, 8, hipMemcpyDeviceToHost));
  if (n) {
    uint32_t uw = (n + 63) / 64;
    uw = (uw + WPB - 1) / WPB * WPB;
    launch_t li = make_launch(ctx, uw, false);
    hipLaunchKernelGGL(k_wait, dim3(uw / WPB), dim3(WG), 0, hs, ctx->d, li, d_tickets, n, d_ptrs);
    HIPCHK(ctx, hipGetLastError());
  }
  s = sync_stream(ctx, hs);
  if (s) return s;
  uint64_t e1 = 0;
  HIPCHK(ctx, hipMemcpy(&e1, ctx->d.cnt + (size_t)C_AUX0 * CSTRIDE, 8, hipMemcpyDeviceToHost));
  return e1 != e0 ? fail(ctx, AGILE_EAGAIN, "wait: some tickets carried EAGAIN") : AGILE_OK;
}

agile_status agile_release(agile_ctx ctx, const agile_ticket* d_tickets, uint32_t n, void* stream) {
  agile_status s = check_usable(ctx);
  if (s) return s;
  if (n == 0) return AGILE_OK;
  if (!d_tickets) return fail(ctx, AGILE_EINVAL, "release: null pointer");
  uint32_t uw = (n + 63) / 64;
  uw = (uw + WPB - 1) / WPB * WPB;
  launch_t li = make_launch(ctx, uw, false);
  hipLaunchKernelGGL(k_release, dim3(uw / WPB), dim3(WG), 0, (hipStream_t)stream, ctx->d, li, d_tickets, n);
  HIPCHK(ctx, hipGetLastError());
  return AGILE_OK;
}

agile_status agile_flush(agile_ctx ctx, agile_store store, void* stream) {
  agile_status s = check_usable(ctx);
  if (s) return s;
  if (store != ctx->store) return fail(ctx, AGILE_EINVAL, "flush: store is not open on this context");
  hipStream_t hs = (hipStream_t)stream;
  uint32_t uw = std::min<uint32_t>((ctx->d.num_lines + 63) / 64, user_wave_cap(ctx, KIND_FLUSH));
  uw = (uw + WPB - 1) / WPB * WPB;
  launch_t li = make_launch(ctx, uw, true);
  hipLaunchKernelGGL(k_flush, dim3(li.service_blocks + uw / WPB), dim3(WG), lds_of(ctx, (const void*)k_flush), hs, ctx->d, li);
  HIPCHK(ctx, hipGetLastError());
  return sync_stream(ctx, hs);
}

agile_status agile_get_stats(agile_ctx ctx, agile_stats* out, int reset) {
  if (!ctx || !out) return AGILE_EINVAL;
  if (ctx->session) return fail(ctx, AGILE_ESTATE, "get_stats: a serving session is open");
  std::vector<uint64_t> c((size_t)C_COUNT * CSTRIDE);
  HIPCHK(ctx, hipDeviceSynchronize());
  HIPCHK(ctx, hipMemcpy(c.data(), ctx->d.cnt, c.size() * 8, hipMemcpyDeviceToHost));
  auto g = [&](uint32_t i) { return c[(size_t)i * CSTRIDE]; };
  // the resident-hit pass counts nothing itself: its requests and hits are the lookups
  // of its launches less those of the bags it deferred
  const uint64_t hit_pass = g(C_HIT_TOTAL) - g(C_DEFLEN);
  out->requests = g(C_REQUESTS) + hit_pass;
  out->hits = g(C_HITS) + hit_pass;
  out->misses = g(C_MISSES);
  out->read_cmds = g(C_READS);
  out->write_cmds = g(C_WRITES);
  out->wb_evict = g(C_WB_EVICT);
  out->wb_flush = g(C_WB_FLUSH);
  out->eagain = g(C_EAGAIN);
  out->sq_spins = g(C_SQ_SPINS);
  out->ctrl_cmds = g(C_CTRL_CMDS);
  out->cq_entries = g(C_CQ_ENTRIES);
  out->submitted = g(C_SUBMITTED);
  out->completed = g(C_COMPLETED);
  out->consumed = g(C_AUX1) + hit_pass;
  out->rows_updated = g(C_WROWS);
  if (reset) {
    const uint32_t keep[] = {C_SUBMITTED, C_COMPLETED, C_USER_DONE, C_WORK, C_SVC_EXIT, C_IMG_EPOCH,
                             C_WORK_P1, C_WORK_P2, C_WORK_P3, C_WORK_P4, C_WORK_P5, C_WORK_P6, C_WORK_P7,
                             C_DEFER};
    for (uint32_t i = 0; i < C_COUNT; ++i) {
      if (std::find(std::begin(keep), std::end(keep), i) != std::end(keep)) continue;
      HIPCHK(ctx, hipMemset(ctx->d.cnt + (size_t)i * CSTRIDE, 0, 8));
    }
    HIPCHK(ctx, hipDeviceSynchronize());
  }
  return AGILE_OK;
}

agile_status agile_set_max_user_waves(agile_ctx ctx, uint32_t n) {
  if (!ctx) return AGILE_EINVAL;
  ctx->cfg.max_user_waves = n;
  return AGILE_OK;
}

agile_status agile_get_info(agile_ctx ctx, agile_info* out) {
  if (!ctx || !out) return AGILE_EINVAL;
  out->num_lines = ctx->d.num_lines;
  out->num_sets = ctx->d.num_sets;
  out->assoc = ctx->d.assoc;
  out->line_bytes = ctx->cfg.line_bytes;
  out->num_qp = ctx->d.num_qp;
  out->qp_depth = ctx->d.depth;
  out->ctrl_waves = ctx->n_ctrl;
  out->cq_waves = ctx->n_cq;
  out->cu_count = ctx->cu_count;
  out->max_user_waves = user_wave_cap(ctx, KIND_EMBBAG2);
  out->wallclock_hz = ctx->clock_hz;
  out->cache_base = (uint64_t)(uintptr_t)ctx->d.lines;
  {
    hipFuncAttributes fa;
    memset(&fa, 0, sizeof(fa));
    const void* f = (const void*)k_embbag<2>;
    const uint32_t st = hipFuncGetAttributes(&fa, f) == hipSuccess ? (uint32_t)fa.sharedSizeBytes : 0u;
    (void)hipGetLastError();
    out->service_lds_bytes = st + lds_of(ctx, f);
  }
  out->service_blocks = ctx->service_blocks;
  return AGILE_OK;
}

// Wavefronts of a fused prefetch launch that prefetch before they compute: enough to keep
// every queue pair's submissions going, few enough that almost every wavefront computes.
constexpr uint32_t PF_WAVES = 64;

static agile_status embbag_launch(agile_ctx ctx, agile_store store, const agile_tables* tb, const int64_t* d_idx,
                                  const int64_t* d_off, uint64_t B, uint64_t n, uint32_t K, uint32_t mode,
                                  float* d_out, void* stream, bool gather, const int64_t* d_next_idx = nullptr,
                                  const int64_t* d_next_off = nullptr, uint64_t B_next = 0) {
  agile_status s = check_usable(ctx);
  if (s) return s;
  if (store != ctx->store) return fail(ctx, AGILE_EINVAL, "workload: store is not open on this context");
  // d_idx may be NULL when every bag is empty (it is only read for existing lookups)
  // (a call that only prefetches, B == 0, needs no output or offsets)
  if (!tb || ((gather || B) && (!d_out || (!gather && !d_off)))) return fail(ctx, AGILE_EINVAL, "workload: null pointer");
  if (tb->dim == 0 || tb->dim > 256 || tb->num_tables == 0 || tb->rows == 0)
    return fail(ctx, AGILE_EINVAL, "workload: dim must be 1..256, tables and rows non-zero");
  const uint64_t row_bytes = (uint64_t)tb->dim * 4;
  if (4096 % row_bytes) return fail(ctx, AGILE_EINVAL, "workload: row bytes must divide 4096");
  if (tb->base_offset % row_bytes) return fail(ctx, AGILE_EINVAL, "workload: base_offset must be row aligned");
  const uint64_t table_bytes = tb->rows * row_bytes;
  if (tb->base_offset + table_bytes * tb->num_tables > store->bytes)
    return fail(ctx, AGILE_EINVAL, "workload: tables exceed the store");
  if (mode > AGILE_MODE_ASYNC) return fail(ctx, AGILE_EINVAL, "workload: bad mode");
  if (B_next && !d_next_off) return fail(ctx, AGILE_EINVAL, "workload: null next-batch offsets");
  embbag_args a{};
  a.idx = d_idx;
  a.off = d_off;
  a.out = d_out;
  a.nbags = gather ? (n + 63) / 64 : B * tb->num_tables;
  a.n = n;
  a.rows = tb->rows;
  a.base_off = tb->base_offset;
  a.table_bytes = table_bytes;
  a.T = tb->num_tables;
  a.dim = tb->dim;
  a.row_bytes = (uint32_t)row_bytes;
  a.K = K;
  a.mode = mode;
  a.gather = gather ? 1u : 0u;
  if (a.nbags == 0 && B_next == 0) return AGILE_OK;
  const int kind = tb->dim <= 64 ? KIND_EMBBAG1 : (tb->dim <= 128 ? KIND_EMBBAG2 : KIND_EMBBAG4);
  uint32_t uw, active;
  if (ctx->cfg.flags & AGILE_F_SERIALIZED) {
    uw = WPB;
    active = 1;
  } else {
    // admission: a wave pins at most two chunks of 64 lines (the current and, in
    // asynchronous mode, the next), and the waves' pins together must fit in the cache;
    // both modes get the same wave count
    const uint64_t by_cache = std::max<uint64_t>(1, ctx->d.num_lines / 128);
    active = (uint32_t)std::min<uint64_t>({a.nbags, (uint64_t)user_wave_cap(ctx, kind), by_cache});
    uw = (active + WPB - 1) / WPB * WPB;
  }
  a.active_waves = active;
  const bool serial = (ctx->cfg.flags & AGILE_F_SERIALIZED) != 0;
  hipStream_t hs = (hipStream_t)stream;
  if (B_next && !serial) {
    // one fused launch: service, the next batch's prefetch and this batch's compute
    // (with its misses served in the same launch); the same admission as the I/O
    // launch, since a computing wave pins at most one chunk of its own misses
    const int pkind = kind - KIND_EMBBAG1 + KIND_PF1;
    const uint64_t by_cache = std::max<uint64_t>(1, ctx->d.num_lines / 128);
    const uint32_t cap = (uint32_t)std::min<uint64_t>(user_wave_cap(ctx, pkind), by_cache);
    pf_args p{};
    p.idx = d_next_idx;
    p.off = d_next_off;
    p.nbags = B_next * tb->num_tables;
    p.store_bytes = store->bytes;
    p.base_off = tb->base_offset;
    p.table_bytes = table_bytes;
    p.row_bytes = (uint32_t)row_bytes;
    p.T = tb->num_tables;
    // a few dedicated prefetch waves when the launch has many; every wave, in turns with
    // its compute, when it has few (a call that only prefetches: up to PF_WAVES waves)
    const bool few = a.nbags && cap <= 4 * PF_WAVES;
    p.waves = few ? cap : std::min<uint32_t>(PF_WAVES, cap);
    p.interleave = few ? 1u : 0u;
    {
      // The backlog: a multiple of the commands the store needs in flight to run at its
      // cap (Little's law: IOPS x latency, over the devices), at most every queue slot.
      // Eight times, at least 2048, with many waves; with few, twice, at least 256: a read
      // that a computing wave misses waits behind the backlog, and with few waves each
      // such wait idles a larger share of the launch.
      const double little = (double)ctx->cfg.iops_cap * (double)ctx->cfg.latency_ns * 1e-9 * ctx->d.n_dev;
      const uint64_t slots = (uint64_t)ctx->cfg.num_qp * ctx->cfg.qp_depth;
      const uint64_t want = few ? std::max<uint64_t>(256, (uint64_t)(2.0 * little))
                                : std::max<uint64_t>(2048, (uint64_t)(8.0 * little));
      p.backlog = std::min<uint64_t>(slots, want);
    }
    embbag_args ap = a;
    ap.mode = AGILE_MODE_ASYNC;
    ap.active_waves = a.nbags ? cap : p.waves;
    const uint32_t puw = (ap.active_waves + WPB - 1) / WPB * WPB;
    const launch_t lp = make_launch(ctx, puw, true);
    const dim3 pg(lp.service_blocks + puw / WPB);
    if (kind == KIND_EMBBAG1)
      hipLaunchKernelGGL(k_embbag_pf<1>, pg, dim3(WG), lds_of(ctx, (const void*)k_embbag_pf<1>), hs, ctx->d, lp, ap, p);
    else if (kind == KIND_EMBBAG2)
      hipLaunchKernelGGL(k_embbag_pf<2>, pg, dim3(WG), lds_of(ctx, (const void*)k_embbag_pf<2>), hs, ctx->d, lp, ap, p);
    else
      hipLaunchKernelGGL(k_embbag_pf<4>, pg, dim3(WG), lds_of(ctx, (const void*)k_embbag_pf<4>), hs, ctx->d, lp, ap, p);
    HIPCHK(ctx, hipGetLastError());
    return AGILE_OK;
  }
  // the resident-hit pass first (see hit_bag), when the deferred list can hold every
  // bag and the wave count is not capped (a cap applies to the I/O launch, which then
  // runs every bag); the I/O launch then runs only the bags the pass deferred.  Both
  // launches are stream ordered; the I/O launch's last service wavefront clears the
  // deferred count, so the pair can be captured in a graph and replayed.
  if (!serial && !ctx->cfg.max_user_waves && a.nbags <= ctx->defer_cap && a.nbags) {
    const dim3 hg((uint32_t)((a.nbags + HIT_WAVES - 1) / HIT_WAVES)), hb(64 * HIT_WAVES);
    if (kind == KIND_EMBBAG1)
      hipLaunchKernelGGL(k_embbag_hit<1>, hg, hb, 0, hs, ctx->d, a, ctx->defer_list);
    else if (kind == KIND_EMBBAG2)
      hipLaunchKernelGGL(k_embbag_hit<2>, hg, hb, 0, hs, ctx->d, a, ctx->defer_list);
    else
      hipLaunchKernelGGL(k_embbag_hit<4>, hg, hb, 0, hs, ctx->d, a, ctx->defer_list);
    HIPCHK(ctx, hipGetLastError());
    a.list = ctx->defer_list;
  }
  if (a.nbags == 0) return AGILE_OK;
  launch_t li = make_launch(ctx, uw, true);
  const dim3 grid(li.service_blocks + uw / WPB);
  if (kind == KIND_EMBBAG1)
    hipLaunchKernelGGL(k_embbag<1>, grid, dim3(WG), lds_of(ctx, (const void*)k_embbag<1>), hs, ctx->d, li, a);
  else if (kind == KIND_EMBBAG2)
    hipLaunchKernelGGL(k_embbag<2>, grid, dim3(WG), lds_of(ctx, (const void*)k_embbag<2>), hs, ctx->d, li, a);
  else
    hipLaunchKernelGGL(k_embbag<4>, grid, dim3(WG), lds_of(ctx, (const void*)k_embbag<4>), hs, ctx->d, li, a);
  HIPCHK(ctx, hipGetLastError());
  return AGILE_OK;
}

agile_status agile_gather(agile_ctx ctx, agile_store store, const agile_tables* tb, const int64_t* d_idx,
                          uint64_t n, uint32_t mode, float* d_out, void* stream) {
  if (n == 0) return check_usable(ctx);
  return embbag_launch(ctx, store, tb, d_idx, nullptr, 0, n, 0, mode, d_out, stream, true);
}

agile_status agile_embbag_forward(agile_ctx ctx, agile_store store, const agile_tables* tb, const int64_t* d_idx,
                                  const int64_t* d_off, uint64_t B, uint32_t K, uint32_t mode, float* d_out,
                                  void* stream) {
  if (B == 0) return check_usable(ctx);
  return embbag_launch(ctx, store, tb, d_idx, d_off, B, 0, K, mode, d_out, stream, false);
}

agile_status agile_embbag_forward_prefetch(agile_ctx ctx, agile_store store, const agile_tables* tb,
                                           const int64_t* d_idx, const int64_t* d_off, uint64_t B, uint32_t K,
                                           float* d_out, const int64_t* d_next_idx, const int64_t* d_next_off,
                                           uint64_t B_next, void* stream) {
  if (B == 0 && B_next == 0) return check_usable(ctx);
  return embbag_launch(ctx, store, tb, d_idx, d_off, B, 0, K, AGILE_MODE_ASYNC, d_out, stream, false,
                       d_next_idx, d_next_off, B_next);
}

agile_status agile_embbag_forward_resident(agile_ctx ctx, const void* d_image, uint64_t image_bytes,
                                           const agile_tables* tb, const int64_t* d_idx, const int64_t* d_off,
                                           uint64_t B, uint32_t K, float* d_out, void* stream) {
  agile_status s = check_usable(ctx);
  if (s) return s;
  if (!tb || !d_image || !d_out || !d_off) return fail(ctx, AGILE_EINVAL, "resident forward: null pointer");
  if (tb->dim == 0 || tb->dim > 256 || tb->num_tables == 0 || tb->rows == 0)
    return fail(ctx, AGILE_EINVAL, "resident forward: dim must be 1..256, tables and rows non-zero");
  const uint64_t row_bytes = (uint64_t)tb->dim * 4;
  if (4096 % row_bytes || tb->base_offset % row_bytes)
    return fail(ctx, AGILE_EINVAL, "resident forward: row bytes must divide 4096 and align base_offset");
  const uint64_t table_bytes = tb->rows * row_bytes;
  if (tb->base_offset + table_bytes * tb->num_tables > image_bytes)
    return fail(ctx, AGILE_EINVAL, "resident forward: tables exceed the image");
  embbag_args a{};
  a.idx = d_idx;
  a.off = d_off;
  a.out = d_out;
  a.nbags = B * tb->num_tables;
  a.rows = tb->rows;
  a.base_off = tb->base_offset;
  a.table_bytes = table_bytes;
  a.T = tb->num_tables;
  a.dim = tb->dim;
  a.row_bytes = (uint32_t)row_bytes;
  a.K = K;
  if (a.nbags == 0) return AGILE_OK;
  if ((a.nbags + RES_WAVES - 1) / RES_WAVES >= (1ull << 31)) return fail(ctx, AGILE_EINVAL, "resident forward: too many bags");
  const dim3 grid((uint32_t)((a.nbags + RES_WAVES - 1) / RES_WAVES)), blk(64 * RES_WAVES);
  const hipStream_t hs = (hipStream_t)stream;
  const uint8_t* img = (const uint8_t*)d_image;
  if (tb->dim <= 64)
    hipLaunchKernelGGL(k_embbag_resident<1>, grid, blk, 0, hs, ctx->d, img, a);
  else if (tb->dim <= 128)
    hipLaunchKernelGGL(k_embbag_resident<2>, grid, blk, 0, hs, ctx->d, img, a);
  else
    hipLaunchKernelGGL(k_embbag_resident<4>, grid, blk, 0, hs, ctx->d, img, a);
  HIPCHK(ctx, hipGetLastError());
  return AGILE_OK;
}

agile_status agile_async_issue(agile_ctx ctx, agile_store store, const uint64_t* d_blocks, uint32_t n,
                               void* const* d_bufs, void** d_ptrs, uint32_t* d_status, uint32_t flags,
                               void* stream) {
  agile_status s = check_usable(ctx);
  if (s) return s;
  if (store != ctx->store) return fail(ctx, AGILE_EINVAL, "async_issue: store is not open on this context");
  if (n == 0) return AGILE_OK;
  if (!d_blocks || !d_bufs || !d_ptrs || !d_status) return fail(ctx, AGILE_EINVAL, "async_issue: null pointer");
  if (flags & ~AGILE_ISSUE_SHARE) return fail(ctx, AGILE_EINVAL, "async_issue: unknown flag");
  hipStream_t hs = (hipStream_t)stream;
  // a wave pins at most one chunk (64 lines) at a time
  const uint64_t by_cache = std::max<uint64_t>(1, ctx->d.num_lines / 64);
  uint32_t uw = (uint32_t)std::min<uint64_t>({(n + 63) / 64, (uint64_t)user_wave_cap(ctx, KIND_ISSUE), by_cache});
  uw = (uw + WPB - 1) / WPB * WPB;
  launch_t li = make_launch(ctx, uw, true);
  hipLaunchKernelGGL(k_async_issue, dim3(li.service_blocks + uw / WPB), dim3(WG),
                     lds_of(ctx, (const void*)k_async_issue), hs, ctx->d, li, d_blocks, n, d_bufs, d_ptrs, d_status,
                     (uint32_t)(flags & AGILE_ISSUE_SHARE));
  HIPCHK(ctx, hipGetLastError());
  return sync_stream(ctx, hs);
}

agile_status agile_buffers_release(agile_ctx ctx, const uint64_t* d_blocks, const uint32_t* d_status, uint32_t n,
                                   void* stream) {
  agile_status s = check_usable(ctx);
  if (s) return s;
  if (n == 0) return AGILE_OK;
  if (!d_blocks || !d_status) return fail(ctx, AGILE_EINVAL, "buffers_release: null pointer");
  hipStream_t hs = (hipStream_t)stream;
  hipLaunchKernelGGL(k_share_release, dim3((n + 255) / 256), dim3(256), 0, hs, ctx->d, d_blocks, d_status, n);
  HIPCHK(ctx, hipGetLastError());
  return sync_stream(ctx, hs);
}

agile_status agile_buffers_writeback(agile_ctx ctx, agile_store store, const uint64_t* d_blocks,
                                     const void* const* d_srcs, uint32_t n, void* stream) {
  agile_status s = check_usable(ctx);
  if (s) return s;
  if (store != ctx->store) return fail(ctx, AGILE_EINVAL, "buffers_writeback: store is not open on this context");
  if (n == 0) return AGILE_OK;
  if (!d_blocks || !d_srcs) return fail(ctx, AGILE_EINVAL, "buffers_writeback: null pointer");
  hipStream_t hs = (hipStream_t)stream;
  const uint64_t by_cache = std::max<uint64_t>(1, ctx->d.num_lines / 64);
  uint32_t uw = (uint32_t)std::min<uint64_t>({(n + 63) / 64, (uint64_t)user_wave_cap(ctx, KIND_WBACK), by_cache});
  uw = (uw + WPB - 1) / WPB * WPB;
  launch_t li = make_launch(ctx, uw, true);
  hipLaunchKernelGGL(k_buf_writeback, dim3(li.service_blocks + uw / WPB), dim3(WG),
                     lds_of(ctx, (const void*)k_buf_writeback), hs, ctx->d, li, d_blocks, n, d_srcs);
  HIPCHK(ctx, hipGetLastError());
  return sync_stream(ctx, hs);
}

agile_status agile_share_reset(agile_ctx ctx) {
  agile_status s = check_usable(ctx);
  if (s) return s;
  HIPCHK(ctx, hipDeviceSynchronize());
  HIPCHK(ctx, hipMemset(ctx->d.share_key, 0, 8ull * SHARE_CAP));
  HIPCHK(ctx, hipMemset(ctx->d.share_refs, 0, 4ull * SHARE_CAP));
  HIPCHK(ctx, hipDeviceSynchronize());
  return AGILE_OK;
}

static agile_status ensure_scratch(agile_ctx ctx, size_t need, hipStream_t hs) {
  if (need <= ctx->scratch_bytes) return AGILE_OK;
  HIPCHK(ctx, hipStreamSynchronize(hs));
  if (ctx->scratch) HIPCHK(ctx, hipFree(ctx->scratch));
  ctx->scratch = nullptr;
  ctx->scratch_bytes = 0;
  if (hipMalloc(&ctx->scratch, need) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, AGILE_ENOMEM, "scratch allocation failed");
  }
  ctx->scratch_bytes = need;
  return AGILE_OK;
}

static agile_status check_csr(agile_ctx ctx, uint64_t bytes, const agile_csr* g, bool need_val) {
  if (!g) return fail(ctx, AGILE_EINVAL, "graph: null csr");
  if (g->num_vertices == 0 || g->num_vertices >= (1ull << 31))
    return fail(ctx, AGILE_EINVAL, "graph: vertex count must be 1..2^31-1");
  if (g->row_ptr_offset % 8 || g->col_offset % 4 || g->val_offset % 4)
    return fail(ctx, AGILE_EINVAL, "graph: misaligned arrays");
  if (g->row_ptr_offset + 8 * (g->num_vertices + 1) > bytes || g->col_offset + 4 * g->num_edges > bytes ||
      (need_val && g->val_offset + 4 * g->num_edges > bytes))
    return fail(ctx, AGILE_EINVAL, "graph: arrays exceed the store");
  return AGILE_OK;
}

static csr_t to_csr(const agile_csr* g) {
  csr_t c;
  c.V = g->num_vertices;
  c.E = g->num_edges;
  c.rp_off = g->row_ptr_offset;
  c.col_off = g->col_offset;
  c.val_off = g->val_offset;
  return c;
}

// Zeroes n 32-bit words (a kernel, so that a captured graph holds no memset node).
__global__ void k_zero32(uint32_t* p, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

__global__ void k_bfs_init(int32_t* level, uint64_t V, uint64_t src, int32_t* F) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < V) level[i] = (i == src) ? 0 : -1;
  if (i == 0) F[0] = (int32_t)src;
}

static agile_status bfs_run(agile_ctx ctx, const agile_csr* g, uint64_t src, int32_t* d_level, uint32_t* out_levels,
                            hipStream_t hs, const uint8_t* img);

agile_status agile_bfs(agile_ctx ctx, agile_store store, const agile_csr* g, uint64_t src, int32_t* d_level,
                       uint32_t* out_levels, void* stream) {
  agile_status s = check_usable(ctx);
  if (s) return s;
  if (store != ctx->store) return fail(ctx, AGILE_EINVAL, "bfs: store is not open on this context");
  if ((s = check_csr(ctx, store->bytes, g, false)) != AGILE_OK) return s;
  if (!d_level || src >= g->num_vertices) return fail(ctx, AGILE_EINVAL, "bfs: bad level array or source");
  return bfs_run(ctx, g, src, d_level, out_levels, (hipStream_t)stream, nullptr);
}

agile_status agile_bfs_resident(agile_ctx ctx, const void* d_image, uint64_t image_bytes, const agile_csr* g,
                                uint64_t src, int32_t* d_level, uint32_t* out_levels, void* stream) {
  agile_status s = check_usable(ctx);
  if (s) return s;
  if (!d_image) return fail(ctx, AGILE_EINVAL, "bfs_resident: null image");
  if ((s = check_csr(ctx, image_bytes, g, false)) != AGILE_OK) return s;
  if (!d_level || src >= g->num_vertices) return fail(ctx, AGILE_EINVAL, "bfs: bad level array or source");
  return bfs_run(ctx, g, src, d_level, out_levels, (hipStream_t)stream, (const uint8_t*)d_image);
}

static agile_status bfs_run(agile_ctx ctx, const agile_csr* g, uint64_t src, int32_t* d_level, uint32_t* out_levels,
                            hipStream_t hs, const uint8_t* img) {
  agile_status s = AGILE_OK;
  const bool svc = img == nullptr;  // a resident image needs no service wavefronts
  const uint64_t V = g->num_vertices;
  const size_t scan_bytes = 8 * sort::scan_work_elems(V);
  auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
  const size_t oF = 0, oN = oF + al(4 * V), ocs = oN + al(4 * V), ocd = ocs + al(8 * V), oco = ocd + al(8 * V),
               octr = oco + al(8 * (V + 1)), osc = octr + 256, need = osc + al(scan_bytes);
  if ((s = ensure_scratch(ctx, need, hs)) != AGILE_OK) return s;
  uint8_t* sb = (uint8_t*)ctx->scratch;
  bfs_args a{};
  a.g = to_csr(g);
  a.img = img;
  a.cs = (uint64_t*)(sb + ocs);
  a.cd = (uint64_t*)(sb + ocd);
  a.co = (uint64_t*)(sb + oco);
  a.ctr = (uint32_t*)(sb + octr);
  a.level = d_level;
  int32_t* F = (int32_t*)(sb + oF);
  int32_t* N = (int32_t*)(sb + oN);
  hipLaunchKernelGGL(k_bfs_init, dim3((uint32_t)((V + 255) / 256)), dim3(256), 0, hs, d_level, V, src, F);
  HIPCHK(ctx, hipGetLastError());
  uint32_t nF = 1;
  int32_t L = 0;
  uint32_t levels = 1;  // levels that hold at least one vertex
  // user waves per level: a 128th of the lines, and at most BFS_MAX_WAVES (past that,
  // more waves walking the edges while the controllers copy make every memory access of
  // the level slower than the extra latency hiding gains: measured on RMAT scale 24 and
  // 26 with 4 and 16 KiB lines, 1536 waves beat both 1024 and the full grid)
  // (a resident image pins no lines: only the cap applies)
  constexpr uint64_t BFS_MAX_WAVES = 1536;
  const uint64_t by_cache =
      img ? BFS_MAX_WAVES : std::max<uint64_t>(1, std::min<uint64_t>(ctx->d.num_lines / 128, BFS_MAX_WAVES));
  while (nF > 0) {
    a.F = F;
    a.N = N;
    a.nF = nF;
    a.L = L;
    hipLaunchKernelGGL(k_zero32, dim3(1), dim3(64), 0, hs, a.ctr, 64u);
    uint32_t uw = (uint32_t)std::min<uint64_t>({(nF + 63) / 64, (uint64_t)user_wave_cap(ctx, KIND_READ), by_cache});
    uw = (uw + WPB - 1) / WPB * WPB;
    launch_t li = make_launch(ctx, uw, svc);
    hipLaunchKernelGGL(k_bfs_front, dim3(li.service_blocks + uw / WPB), dim3(WG), lds_of(ctx, (const void*)k_bfs_front), hs, ctx->d, li, a);
    HIPCHK(ctx, hipGetLastError());
    uint32_t nC = 0;
    HIPCHK(ctx, hipMemcpyAsync(&nC, a.ctr, 4, hipMemcpyDeviceToHost, hs));
    if ((s = sync_stream(ctx, hs)) != AGILE_OK) return s;
    if (nC == 0) break;
    if (!sort::exclusive_scan<uint64_t>(a.cd, a.co, nC, (uint64_t*)(sb + osc), hs))
      return fail(ctx, AGILE_EHIP, std::string("bfs: scan launch failed: ") + hipGetErrorString(hipGetLastError()));
    uint64_t last[2] = {0, 0};
    HIPCHK(ctx, hipMemcpyAsync(&last[0], a.co + nC - 1, 8, hipMemcpyDeviceToHost, hs));
    HIPCHK(ctx, hipMemcpyAsync(&last[1], a.cd + nC - 1, 8, hipMemcpyDeviceToHost, hs));
    HIPCHK(ctx, hipStreamSynchronize(hs));
    a.nC = nC;
    a.Et = last[0] + last[1];
    uw = (uint32_t)std::min<uint64_t>({(a.Et + 1023) / 1024, (uint64_t)user_wave_cap(ctx, KIND_READ), by_cache});
    uw = (uw + WPB - 1) / WPB * WPB;
    li = make_launch(ctx, uw, svc);
    hipLaunchKernelGGL(k_bfs_edges, dim3(li.service_blocks + uw / WPB), dim3(WG), lds_of(ctx, (const void*)k_bfs_edges), hs, ctx->d, li, a);
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, hipMemcpyAsync(&nF, a.ctr + 1, 4, hipMemcpyDeviceToHost, hs));
    if ((s = sync_stream(ctx, hs)) != AGILE_OK) return s;
    if (nF) ++levels;
    std::swap(F, N);
    ++L;
  }
  if (out_levels) *out_levels = levels;
  return AGILE_OK;
}

static agile_status spmv_run(agile_ctx ctx, const agile_csr* g, const float* d_x, float* d_y, hipStream_t hs,
                             const uint8_t* img);

agile_status agile_spmv(agile_ctx ctx, agile_store store, const agile_csr* g, const float* d_x, float* d_y,
                        void* stream) {
  agile_status s = check_usable(ctx);
  if (s) return s;
  if (store != ctx->store) return fail(ctx, AGILE_EINVAL, "spmv: store is not open on this context");
  if ((s = check_csr(ctx, store->bytes, g, true)) != AGILE_OK) return s;
  if (!d_x || !d_y) return fail(ctx, AGILE_EINVAL, "spmv: null vector");
  return spmv_run(ctx, g, d_x, d_y, (hipStream_t)stream, nullptr);
}

agile_status agile_spmv_resident(agile_ctx ctx, const void* d_image, uint64_t image_bytes, const agile_csr* g,
                                 const float* d_x, float* d_y, void* stream) {
  agile_status s = check_usable(ctx);
  if (s) return s;
  if (!d_image) return fail(ctx, AGILE_EINVAL, "spmv_resident: null image");
  if ((s = check_csr(ctx, image_bytes, g, true)) != AGILE_OK) return s;
  if (!d_x || !d_y) return fail(ctx, AGILE_EINVAL, "spmv: null vector");
  return spmv_run(ctx, g, d_x, d_y, (hipStream_t)stream, (const uint8_t*)d_image);
}

static agile_status spmv_run(agile_ctx ctx, const agile_csr* g, const float* d_x, float* d_y, hipStream_t hs,
                             const uint8_t* img) {
  spmv_args a{};
  a.g = to_csr(g);
  a.img = img;
  a.x = d_x;
  a.y = d_y;
  // a wave pins at most two windows (the current one and the prefetch) of 2 x 8 lines; a
  // resident image pins none
  const uint64_t by_cache = img ? UINT64_MAX : std::max<uint64_t>(1, ctx->d.num_lines / 32);
  const uint32_t active = (uint32_t)std::min<uint64_t>(
      {(g->num_vertices + 64 * SPMV_RUN - 1) / (64 * SPMV_RUN), (uint64_t)user_wave_cap(ctx, KIND_READ), by_cache});
  a.active = std::max<uint32_t>(1, active);
  const uint32_t uw = (a.active + WPB - 1) / WPB * WPB;
  // without service wavefronts nobody clears the launch's work counter on exit: clear it
  // before and after the launch
  uint32_t* work = reinterpret_cast<uint32_t*>(ctx->d.cnt + (size_t)C_WORK * CSTRIDE);
  if (img) hipLaunchKernelGGL(k_zero32, dim3(1), dim3(64), 0, hs, work, 2u);
  launch_t li = make_launch(ctx, uw, img == nullptr);
  hipLaunchKernelGGL(k_spmv, dim3(li.service_blocks + uw / WPB), dim3(WG), lds_of(ctx, (const void*)k_spmv), hs, ctx->d, li, a);
  HIPCHK(ctx, hipGetLastError());
  if (img) hipLaunchKernelGGL(k_zero32, dim3(1), dim3(64), 0, hs, work, 2u);
  return AGILE_OK;
}


static agile_status bwd_launch(agile_ctx ctx, const agile_tables* tb, const int64_t* d_idx, const int64_t* d_off,
                               uint64_t B, uint64_t n, const float* d_grad, float lr, void* work, hipStream_t hs,
                               const int64_t* d_next_idx = nullptr, const int64_t* d_next_off = nullptr,
                               uint64_t B_next = 0);

// Argument checks shared by both backward entry points (nothing is launched on failure).
static agile_status bwd_check(agile_ctx ctx, agile_store store, const agile_tables* tb, const int64_t* d_idx,
                              const int64_t* d_off, uint64_t n, const float* d_grad) {
  if (store != ctx->store) return fail(ctx, AGILE_EINVAL, "backward: store is not open on this context");
  if (!tb || !d_off || !d_grad || (n && !d_idx)) return fail(ctx, AGILE_EINVAL, "backward: null pointer");
  if (tb->dim == 0 || tb->dim > 256 || tb->num_tables == 0 || tb->rows == 0)
    return fail(ctx, AGILE_EINVAL, "backward: dim must be 1..256, tables and rows non-zero");
  const uint64_t row_bytes = (uint64_t)tb->dim * 4;
  if (4096 % row_bytes || tb->base_offset % row_bytes)
    return fail(ctx, AGILE_EINVAL, "backward: row bytes must divide 4096 and align base_offset");
  if (tb->base_offset + tb->rows * row_bytes * tb->num_tables > store->bytes)
    return fail(ctx, AGILE_EINVAL, "backward: tables exceed the store");
  if (n >= (1ull << 32) || tb->rows * tb->num_tables >= (1ull << 32))
    return fail(ctx, AGILE_EINVAL, "backward: too many lookups or rows");
  return AGILE_OK;
}

agile_status agile_embbag_backward_sgd(agile_ctx ctx, agile_store store, const agile_tables* tb,
                                       const int64_t* d_idx, const int64_t* d_off, uint64_t B, uint64_t n,
                                       const float* d_grad, float lr, void* stream) {
  agile_status s = check_usable(ctx);
  if (s) return s;
  if ((s = bwd_check(ctx, store, tb, d_idx, d_off, n, d_grad)) != AGILE_OK) return s;
  if (n == 0 || B == 0) return AGILE_OK;
  hipStream_t hs = (hipStream_t)stream;
  const size_t need = bwd_work_bytes(n);
  if ((s = ensure_scratch(ctx, need, hs)) != AGILE_OK) return s;
  return bwd_launch(ctx, tb, d_idx, d_off, B, n, d_grad, lr, ctx->scratch, hs);
}

agile_status agile_embbag_backward_sgd_prefetch(agile_ctx ctx, agile_store store, const agile_tables* tb,
                                                const int64_t* d_idx, const int64_t* d_off, uint64_t B, uint64_t n,
                                                const float* d_grad, float lr, const int64_t* d_next_idx,
                                                const int64_t* d_next_off, uint64_t B_next, void* stream) {
  agile_status s = check_usable(ctx);
  if (s) return s;
  if ((s = bwd_check(ctx, store, tb, d_idx, d_off, n, d_grad)) != AGILE_OK) return s;
  if (B_next && !d_next_off) return fail(ctx, AGILE_EINVAL, "backward: null next-batch offsets");
  if (ctx->cfg.flags & AGILE_F_SERIALIZED) B_next = 0;
  hipStream_t hs = (hipStream_t)stream;
  if (n == 0 || B == 0) {
    // nothing to update: the prefetch alone, as agile_embbag_forward_prefetch does it
    if (!B_next) return AGILE_OK;
    return embbag_launch(ctx, store, tb, nullptr, nullptr, 0, 0, 0, AGILE_MODE_ASYNC, nullptr, stream, false,
                         d_next_idx, d_next_off, B_next);
  }
  const size_t need = bwd_work_bytes(n);
  if ((s = ensure_scratch(ctx, need, hs)) != AGILE_OK) return s;
  return bwd_launch(ctx, tb, d_idx, d_off, B, n, d_grad, lr, ctx->scratch, hs, d_next_idx, d_next_off, B_next);
}

agile_status agile_embbag_backward_sgd_noalloc(agile_ctx ctx, agile_store store, const agile_tables* tb,
                                               const int64_t* d_idx, const int64_t* d_off, uint64_t B,
                                               uint64_t n, const float* d_grad, float lr, void* stream) {
  agile_status s = check_usable(ctx);
  if (s) return s;
  if ((s = bwd_check(ctx, store, tb, d_idx, d_off, n, d_grad)) != AGILE_OK) return s;
  if (n > NOALLOC_MAX_LOOKUPS)
    return fail(ctx, AGILE_EINVAL,
                "backward_noalloc: " + std::to_string(n) + " lookups exceed the fixed work area's maximum of " +
                    std::to_string(NOALLOC_MAX_LOOKUPS));
  if (n == 0 || B == 0) return AGILE_OK;
  if (!ctx->noalloc_scratch) return fail(ctx, AGILE_ESTATE, "backward_noalloc: no work area on this device");
  return bwd_launch(ctx, tb, d_idx, d_off, B, n, d_grad, lr, ctx->noalloc_scratch, (hipStream_t)stream);
}

static agile_status bwd_launch(agile_ctx ctx, const agile_tables* tb, const int64_t* d_idx, const int64_t* d_off,
                               uint64_t B, uint64_t n, const float* d_grad, float lr, void* work, hipStream_t hs,
                               const int64_t* d_next_idx, const int64_t* d_next_off, uint64_t B_next) {
  const uint64_t nbags = B * tb->num_tables;
  const uint64_t row_bytes = (uint64_t)tb->dim * 4;
  uint8_t* sb = (uint8_t*)work;
  const size_t o_keys = 0, o_bag = o_keys + bwd_al(n * 8), o_head = o_bag + bwd_al(n * 4),
               o_ctr = o_head + bwd_al(n * 4), o_sort = o_ctr + 256;
  bwd_args a{};
  a.idx = d_idx;
  a.off = d_off;
  a.grad = d_grad;
  a.bagid = (uint32_t*)(sb + o_bag);
  a.heads = (uint32_t*)(sb + o_head);
  a.ctr = (uint32_t*)(sb + o_ctr);
  a.n = n;
  a.nbags = nbags;
  a.rows = tb->rows;
  a.base_off = tb->base_offset;
  a.T = tb->num_tables;
  a.dim = tb->dim;
  a.row_bytes = (uint32_t)row_bytes;
  a.lr = lr;
  hipLaunchKernelGGL(k_zero32, dim3(1), dim3(64), 0, hs, a.ctr, 64u);
  uint64_t* keys_in = (uint64_t*)(sb + o_keys);
  hipLaunchKernelGGL(k_bwd_keys, dim3((uint32_t)((nbags + 255) / 256)), dim3(256), 0, hs, a, keys_in);
  HIPCHK(ctx, hipGetLastError());
  // the keys are written in ascending lookup position, so a stable sort by the row bits
  // alone leaves every row's occurrences in ascending position
  const uint32_t row_bits = log2u(tb->rows * tb->num_tables);
  uint64_t* sorted = nullptr;
  if (!sort::radix_sort(keys_in, n, 32, 32 + std::max<uint32_t>(row_bits, 1), sb + o_sort, hs, &sorted))
    return fail(ctx, AGILE_EHIP, std::string("backward: sort launch failed: ") + hipGetErrorString(hipGetLastError()));
  a.keys = sorted;
  hipLaunchKernelGGL(k_bwd_heads, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, hs, a);
  HIPCHK(ctx, hipGetLastError());
  const int kind = tb->dim <= 64 ? KIND_BWD1 : (tb->dim <= 128 ? KIND_BWD2 : KIND_BWD4);
  const uint64_t by_cache = std::max<uint64_t>(1, ctx->d.num_lines / 128);
  uint32_t uw = (uint32_t)std::min<uint64_t>({(n + 63) / 64, (uint64_t)user_wave_cap(ctx, kind), by_cache});
  uw = (uw + WPB - 1) / WPB * WPB;
  launch_t li = make_launch(ctx, uw, true);
  const dim3 grid(li.service_blocks + uw / WPB);
  pf_args p{};
  if (B_next) {
    // the next batch's prefetch rides on this launch's leading waves (as in the forward's
    // fused launch with many waves: a few prefetch, the rest never stop computing)
    p.idx = d_next_idx;
    p.off = d_next_off;
    p.nbags = B_next * tb->num_tables;
    p.store_bytes = ctx->store->bytes;
    p.base_off = tb->base_offset;
    p.table_bytes = tb->rows * row_bytes;
    p.row_bytes = (uint32_t)row_bytes;
    p.T = tb->num_tables;
    p.waves = std::min<uint32_t>(PF_WAVES, uw);
    const double little = (double)ctx->cfg.iops_cap * (double)ctx->cfg.latency_ns * 1e-9 * ctx->d.n_dev;
    const uint64_t slots = (uint64_t)ctx->cfg.num_qp * ctx->cfg.qp_depth;
    p.backlog = std::min<uint64_t>(slots, std::max<uint64_t>(2048, (uint64_t)(8.0 * little)));
  }
  if (kind == KIND_BWD1)
    hipLaunchKernelGGL(k_bwd_sgd<1>, grid, dim3(WG), lds_of(ctx, (const void*)k_bwd_sgd<1>), hs, ctx->d, li, a, p);
  else if (kind == KIND_BWD2)
    hipLaunchKernelGGL(k_bwd_sgd<2>, grid, dim3(WG), lds_of(ctx, (const void*)k_bwd_sgd<2>), hs, ctx->d, li, a, p);
  else
    hipLaunchKernelGGL(k_bwd_sgd<4>, grid, dim3(WG), lds_of(ctx, (const void*)k_bwd_sgd<4>), hs, ctx->d, li, a, p);
  HIPCHK(ctx, hipGetLastError());
  return AGILE_OK;
}

agile_status agile_probe_copy(const void* src, const uint64_t* d_list, uint64_t n, void* d_dst, uint64_t dst_blocks,
                              uint32_t waves, uint32_t per_wave, void* stream) {
  if (!src || !d_dst || n == 0 || dst_blocks == 0 || waves == 0 || per_wave == 0 || per_wave > 4)
    return AGILE_EINVAL;
  hipPointerAttribute_t attr;
  memset(&attr, 0, sizeof(attr));
  const uint8_t* s = (const uint8_t*)src;
  if (hipPointerGetAttributes(&attr, src) == hipSuccess && attr.type == hipMemoryTypeHost && attr.devicePointer)
    s = (const uint8_t*)attr.devicePointer + ((const uint8_t*)src - (const uint8_t*)attr.hostPointer);
  (void)hipGetLastError();
  const uint32_t blocks = (waves + WPB - 1) / WPB;
  hipLaunchKernelGGL(k_probe_copy, dim3(blocks), dim3(WG), 0, (hipStream_t)stream, s, d_list, n, (uint8_t*)d_dst,
                     dst_blocks, per_wave);
  return hipGetLastError() == hipSuccess ? AGILE_OK : AGILE_EHIP;
}

// ---- lock-chain walker on a given wait state (diagnostics)
__global__ void k_lc_walk(dev_ctx c, uint32_t n_waits, uint32_t w0, uint64_t what) {
  // the given waits are current: stamp them now
  for (uint32_t w = threadIdx.x; w < n_waits; w += 64)
    if (ld_rlx(c.waits + 2 * w)) st_rlx(c.waits + 2 * w + 1, now());
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  if (threadIdx.x == 0) lc_walk(c, w0, what);
}

agile_status agile_debug_lockchain(agile_ctx ctx, const uint64_t* waits, uint32_t n_waits, const uint32_t* lock_sets,
                                   const uint32_t* lock_words, uint32_t n_locks, uint32_t start_wave,
                                   uint64_t start_what, char* msg, uint32_t msg_len) {
  agile_status s = check_usable(ctx);
  if (s) return s;
  if ((n_waits && !waits) || (n_locks && (!lock_sets || !lock_words)) || !msg || !msg_len)
    return fail(ctx, AGILE_EINVAL, "lockchain: null pointer");
  if (n_waits > WAIT_SLOTS || start_wave >= WAIT_SLOTS) return fail(ctx, AGILE_EINVAL, "lockchain: wave out of range");
  for (uint32_t i = 0; i < n_locks; ++i)
    if (lock_sets[i] >= ctx->d.num_sets) return fail(ctx, AGILE_EINVAL, "lockchain: set out of range");
  HIPCHK(ctx, hipDeviceSynchronize());
  if (n_waits) {
    std::vector<uint64_t> w2(2ull * n_waits, 0);
    for (uint32_t i = 0; i < n_waits; ++i) w2[2 * i] = waits[i];
    HIPCHK(ctx, hipMemcpy(ctx->d.waits, w2.data(), 16ull * n_waits, hipMemcpyHostToDevice));
  }
  for (uint32_t i = 0; i < n_locks; ++i)
    HIPCHK(ctx, hipMemcpy(ctx->d.set_lock + lock_sets[i], lock_words + i, 4, hipMemcpyHostToDevice));
  HIPCHK(ctx, hipMemset(ctx->d.chain, 0, 8ull * (1 + 3 * LC_MAX) + 8));
  hipLaunchKernelGGL(k_lc_walk, dim3(1), dim3(64), 0, nullptr, ctx->d, n_waits, start_wave, start_what);
  HIPCHK(ctx, hipGetLastError());
  HIPCHK(ctx, hipDeviceSynchronize());
  std::vector<uint64_t> ch(1 + 3 * LC_MAX + 1, 0);
  HIPCHK(ctx, hipMemcpy(ch.data(), ctx->d.chain, ch.size() * 8, hipMemcpyDeviceToHost));
  // put the state back: no wait recorded, the given set locks free, no chain
  if (n_waits) HIPCHK(ctx, hipMemset(ctx->d.waits, 0, 16ull * n_waits));
  for (uint32_t i = 0; i < n_locks; ++i) HIPCHK(ctx, hipMemset(ctx->d.set_lock + lock_sets[i], 0, 4));
  HIPCHK(ctx, hipMemset(ctx->d.chain, 0, 8ull * (1 + 3 * LC_MAX) + 8));
  HIPCHK(ctx, hipDeviceSynchronize());
  const std::string t = format_chain(ch.data());
  snprintf(msg, msg_len, "%s", t.size() > 2 ? t.c_str() + 2 : "");
  return AGILE_OK;
}

// ---- serving sessions: one persistent kernel fed through rings in pinned host memory
static uint64_t pow2_at_least(uint64_t v) {
  uint64_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

agile_status agile_session_open(agile_ctx ctx, agile_store store, const agile_tables* tb, uint32_t K, uint32_t mode,
                                const agile_serve_opts* opts, agile_session* out) {
  agile_status s = check_usable(ctx);
  if (s) return s;
  if (!out) return fail(ctx, AGILE_EINVAL, "session: null handle");
  *out = nullptr;
  if (ctx->session) return fail(ctx, AGILE_ESTATE, "session: one session per context at a time");
  if (store != ctx->store) return fail(ctx, AGILE_EINVAL, "session: store is not open on this context");
  if (!tb || tb->dim == 0 || tb->dim > 256 || 4096 % (tb->dim * 4) || tb->num_tables == 0 || tb->rows == 0)
    return fail(ctx, AGILE_EINVAL, "session: bad tables");
  if (mode > AGILE_MODE_ASYNC) return fail(ctx, AGILE_EINVAL, "session: bad mode");
  const uint64_t row_bytes = (uint64_t)tb->dim * 4, table_bytes = tb->rows * row_bytes;
  if (tb->base_offset % row_bytes || tb->base_offset + table_bytes * tb->num_tables > store->bytes)
    return fail(ctx, AGILE_EINVAL, "session: tables exceed the store");
  agile_session_s* se = new agile_session_s();
  se->ctx = ctx;
  se->tb = *tb;
  const uint64_t sq_slots = (uint64_t)ctx->d.num_qp * ctx->d.depth;
  se->cap_look = opts && opts->max_inflight_lookups ? opts->max_inflight_lookups : sq_slots;
  se->cap_lines = opts && opts->max_inflight_lines ? opts->max_inflight_lines : std::max<uint64_t>(1, ctx->d.num_lines);
  se->cap_req = opts && opts->max_inflight_requests ? opts->max_inflight_requests : 4096;
  // rings: room for what the budgets admit, plus one request of the largest size
  // (ring sizes are bounded; budgets beyond them are limited by ring room instead)
  const uint64_t ring_look = std::min<uint64_t>(std::max<uint64_t>(se->cap_look, 1), 1ull << 22);
  se->look_cap = pow2_at_least(ring_look + SESSION_MAX_LOOKUPS);
  se->bag_cap = pow2_at_least(ring_look + SESSION_MAX_LOOKUPS);
  se->req_cap = pow2_at_least(std::min<uint64_t>(se->cap_req, 1ull << 20) + 1);
  auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
  const size_t o_ctl = 0, o_j0 = o_ctl + 256, o_j1 = o_j0 + al(8 * se->bag_cap), o_breq = o_j1 + al(8 * se->bag_cap),
               o_btab = o_breq + al(8 * se->bag_cap), o_idx = o_btab + al(4 * se->bag_cap),
               o_rnb = o_idx + al(8 * se->look_cap), o_done = o_rnb + al(4 * se->req_cap),
               o_out = o_done + al(4 * se->req_cap), hbytes = o_out + al(4 * se->bag_cap * tb->dim);
  auto cleanup = [&](agile_status st, const std::string& msg) {
    if (se->host) (void)hipHostFree(se->host);
    if (se->dev) (void)hipFree(se->dev);
    if (se->hs) (void)hipStreamDestroy(se->hs);
    delete se;
    return fail(ctx, st, msg);
  };
  if (hipHostMalloc(&se->host, hbytes, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
    (void)hipGetLastError();
    se->host = nullptr;
    return cleanup(AGILE_ENOMEM, "session: pinned ring allocation failed");
  }
  memset(se->host, 0, hbytes);
  uint8_t* hb = (uint8_t*)se->host;
  se->ctl = (uint64_t*)(hb + o_ctl);
  se->bag_j0 = (uint64_t*)(hb + o_j0);
  se->bag_j1 = (uint64_t*)(hb + o_j1);
  se->bag_req = (uint64_t*)(hb + o_breq);
  se->bag_tab = (uint32_t*)(hb + o_btab);
  se->idx = (int64_t*)(hb + o_idx);
  se->req_nbags = (uint32_t*)(hb + o_rnb);
  se->done = (uint32_t*)(hb + o_done);
  se->out = (float*)(hb + o_out);
  void* dhb = nullptr;
  if (hipHostGetDevicePointer(&dhb, se->host, 0) != hipSuccess) return cleanup(AGILE_EHIP, "session: mapping");
  uint8_t* dh = (uint8_t*)dhb;
  // HBM: per-request-slot bag counters, the staged count and stop flag, and the HBM
  // copies of the rings that the waves read
  const size_t q_cnt = 0, q_pub = q_cnt + al(4 * se->req_cap), q_j0 = q_pub + 256,
               q_j1 = q_j0 + al(8 * se->bag_cap), q_req = q_j1 + al(8 * se->bag_cap),
               q_tab = q_req + al(8 * se->bag_cap), q_rnb = q_tab + al(4 * se->bag_cap),
               q_idx = q_rnb + al(4 * se->req_cap), dbytes = q_idx + al(8 * se->look_cap);
  if (hipMalloc(&se->dev, dbytes) != hipSuccess) {
    (void)hipGetLastError();
    se->dev = nullptr;
    return cleanup(AGILE_ENOMEM, "session: device allocation failed");
  }
  if (hipMemset(se->dev, 0, dbytes) != hipSuccess) return cleanup(AGILE_EHIP, "session: memset");
  if (hipStreamCreateWithFlags(&se->hs, hipStreamNonBlocking) != hipSuccess) {
    se->hs = nullptr;
    return cleanup(AGILE_EHIP, "session: stream");
  }
  uint8_t* db = (uint8_t*)se->dev;
  serve_stage sg{};
  sg.h_j0 = (const uint64_t*)(dh + o_j0);
  sg.h_j1 = (const uint64_t*)(dh + o_j1);
  sg.h_req = (const uint64_t*)(dh + o_breq);
  sg.h_tab = (const uint32_t*)(dh + o_btab);
  sg.h_rnb = (const uint32_t*)(dh + o_rnb);
  sg.h_idx = (const int64_t*)(dh + o_idx);
  sg.d_j0 = (uint64_t*)(db + q_j0);
  sg.d_j1 = (uint64_t*)(db + q_j1);
  sg.d_req = (uint64_t*)(db + q_req);
  sg.d_tab = (uint32_t*)(db + q_tab);
  sg.d_rnb = (uint32_t*)(db + q_rnb);
  sg.d_idx = (int64_t*)(db + q_idx);
  sg.pub_dev = (uint64_t*)(db + q_pub);
  embbag_args a{};
  a.idx = sg.d_idx;
  a.out = (float*)(dh + o_out);
  a.nbags = (uint64_t)INT64_MAX;  // an unbounded stream: the session ends on the stop flag
  a.rows = tb->rows;
  a.base_off = tb->base_offset;
  a.table_bytes = table_bytes;
  a.T = tb->num_tables;
  a.dim = tb->dim;
  a.row_bytes = (uint32_t)row_bytes;
  a.K = K;
  a.mode = mode;
  a.serve = 1;
  a.bag_j0 = sg.d_j0;
  a.bag_j1 = sg.d_j1;
  a.bag_req = sg.d_req;
  a.bag_tab = sg.d_tab;
  a.req_nbags = sg.d_rnb;
  a.done = (uint32_t*)(dh + o_done);
  a.req_cnt = (uint32_t*)(db + q_cnt);
  a.pub_dev = sg.pub_dev;
  a.pub_host = (const uint64_t*)(dh + o_ctl);
  a.bag_mask = se->bag_cap - 1;
  a.look_mask = se->look_cap - 1;
  a.req_mask = se->req_cap - 1;
  const int kind = tb->dim <= 64 ? KIND_SERVE1 : (tb->dim <= 128 ? KIND_SERVE2 : KIND_SERVE4);
  // default: a sixteenth of the lines in waves; an explicit count overrides that (the
  // EAGAIN drain keeps an over-subscribed cache deadlock-free, only slower)
  const uint64_t by_cache = std::max<uint64_t>(1, ctx->d.num_lines / 16);
  const uint64_t want = opts && opts->user_waves ? opts->user_waves : by_cache;
  const uint32_t svc_blocks = service_blocks_for(ctx->n_ctrl + ctx->n_cq + 1);  // + the publication mirror
  const uint32_t active =
      (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(want, (uint64_t)user_wave_cap(ctx, kind, svc_blocks)));
  const uint32_t uw = (active + WPB - 1) / WPB * WPB;
  a.active_waves = active;
  se->user_waves = active;
  launch_t li = make_launch(ctx, uw, true);
  li.service_blocks = svc_blocks;
  const dim3 grid(li.service_blocks + uw / WPB);
  if (kind == KIND_SERVE1)
    hipLaunchKernelGGL(k_serve<1>, grid, dim3(WG), lds_of(ctx, (const void*)k_serve<1>), se->hs, ctx->d, li, a, sg);
  else if (kind == KIND_SERVE2)
    hipLaunchKernelGGL(k_serve<2>, grid, dim3(WG), lds_of(ctx, (const void*)k_serve<2>), se->hs, ctx->d, li, a, sg);
  else
    hipLaunchKernelGGL(k_serve<4>, grid, dim3(WG), lds_of(ctx, (const void*)k_serve<4>), se->hs, ctx->d, li, a, sg);
  if (hipGetLastError() != hipSuccess) return cleanup(AGILE_EHIP, "session: launch failed");
  ctx->session = se;
  *out = se;
  return AGILE_OK;
}

agile_status agile_session_submit(agile_session se, uint32_t nbags, const int64_t* bag_off, const int64_t* idx,
                                  uint64_t* out_req) {
  if (!se) return AGILE_EINVAL;
  agile_ctx ctx = se->ctx;
  if (ctx->poisoned || *ctx->abort_host) return map_device_error(ctx) ? map_device_error(ctx) : AGILE_ETIMEDOUT;
  if (!bag_off || !out_req || nbags == 0 || bag_off[0] != 0)
    return fail(ctx, AGILE_EINVAL, "submit: a request needs >= 1 bag and offsets from 0");
  for (uint32_t k = 0; k < nbags; ++k)
    if (bag_off[k + 1] < bag_off[k]) return fail(ctx, AGILE_EINVAL, "submit: bag offsets must not decrease");
  const uint64_t L = (uint64_t)bag_off[nbags];
  if (L && !idx) return fail(ctx, AGILE_EINVAL, "submit: null lookups");
  if (L > SESSION_MAX_LOOKUPS || nbags > SESSION_MAX_LOOKUPS)
    return fail(ctx, AGILE_EINVAL, "submit: request larger than the session's maximum");
  for (uint64_t j = 0; j < L; ++j)
    if (idx[j] < 0 || (uint64_t)idx[j] >= se->tb.rows) return fail(ctx, AGILE_EINVAL, "submit: row out of range");
  // admission: the queue budget (lookups in flight, each may miss), the cache budget (the
  // lines one chunk of each request in flight can pin), the request budget, ring room
  const uint64_t lines = std::min<uint64_t>({std::max<uint64_t>(L, 1), (uint64_t)64,
                                             std::max<uint64_t>(1, se->cap_lines / 2)});
  const bool empty = se->live.empty();
  if (!empty && (se->in_look + L > se->cap_look || se->in_lines + lines > se->cap_lines ||
                 se->live.size() >= se->cap_req))
    return AGILE_EAGAIN;
  const uint64_t bag_tail = empty ? se->next_bag : se->live.front().bag0;
  const uint64_t look_tail = empty ? se->next_look : se->live.front().look0;
  const uint64_t req_tail = empty ? se->next_req : se->live.front().id;
  if (se->next_bag + nbags - bag_tail > se->bag_cap || se->next_look + L - look_tail > se->look_cap ||
      se->next_req + 1 - req_tail > se->req_cap)
    return AGILE_EAGAIN;
  const uint64_t r = se->next_req, b0 = se->next_bag, j0 = se->next_look;
  for (uint32_t k = 0; k < nbags; ++k) {
    const uint64_t slot = (b0 + k) & (se->bag_cap - 1);
    se->bag_j0[slot] = j0 + (uint64_t)bag_off[k];
    se->bag_j1[slot] = j0 + (uint64_t)bag_off[k + 1];
    se->bag_req[slot] = r;
    se->bag_tab[slot] = k % se->tb.num_tables;
  }
  for (uint64_t j = 0; j < L; ++j) se->idx[(j0 + j) & (se->look_cap - 1)] = idx[j];
  const uint64_t rs = r & (se->req_cap - 1);
  se->req_nbags[rs] = nbags;
  __atomic_store_n(&se->done[rs], 0u, __ATOMIC_RELAXED);
  // publication: every entry above is written before the count that makes it visible
  __atomic_store_n(&se->ctl[0], b0 + nbags, __ATOMIC_RELEASE);
  se->live.push_back({r, b0, nbags, j0, L, lines, false});
  se->next_req = r + 1;
  se->next_bag = b0 + nbags;
  se->next_look = j0 + L;
  se->in_look += L;
  se->in_lines += lines;
  *out_req = r;
  return AGILE_OK;
}

agile_status agile_session_poll(agile_session se, uint64_t req, float* out) {
  if (!se) return AGILE_EINVAL;
  agile_ctx ctx = se->ctx;
  if (se->live.empty() || req < se->live.front().id || req >= se->next_req)
    return fail(ctx, AGILE_EINVAL, "poll: unknown or already collected request");
  session_req& e = se->live[req - se->live.front().id];
  if (e.polled) return fail(ctx, AGILE_EINVAL, "poll: request already collected");
  if (!__atomic_load_n(&se->done[req & (se->req_cap - 1)], __ATOMIC_ACQUIRE)) {
    if (*ctx->abort_host) {
      ctx->poisoned = true;
      return fail(ctx, AGILE_ETIMEDOUT, "poll: the session was aborted on the device");
    }
    return AGILE_EAGAIN;
  }
  const uint32_t dim = se->tb.dim;
  if (out)
    for (uint64_t k = 0; k < e.nb; ++k)
      memcpy(out + k * dim, se->out + ((e.bag0 + k) & (se->bag_cap - 1)) * dim, 4ull * dim);
  e.polled = true;
  se->in_look -= e.nl;
  se->in_lines -= e.lines;
  while (!se->live.empty() && se->live.front().polled) se->live.pop_front();
  return AGILE_OK;
}

agile_status agile_session_close(agile_session se) {
  if (!se) return AGILE_EINVAL;
  agile_ctx ctx = se->ctx;
  // every request already submitted completes first (outputs not collected are dropped)
  const double limit_s = 4.0 * (double)ctx->cfg.timeout_ns * 1e-9 + 30.0;
  const auto t0 = std::chrono::steady_clock::now();
  agile_status st = AGILE_OK;
  for (const session_req& e : se->live) {
    while (!e.polled && !__atomic_load_n(&se->done[e.id & (se->req_cap - 1)], __ATOMIC_ACQUIRE)) {
      if (*ctx->abort_host ||
          std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() > limit_s) {
        __atomic_store_n(ctx->abort_host, 1u, __ATOMIC_SEQ_CST);
        st = fail(ctx, AGILE_ETIMEDOUT, "session close: requests did not complete");
        break;
      }
      std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
    if (st != AGILE_OK) break;
  }
  __atomic_store_n(&se->ctl[1], 1ull, __ATOMIC_RELEASE);  // stop
  const agile_status s2 = sync_stream(ctx, se->hs);
  (void)hipStreamDestroy(se->hs);
  (void)hipFree(se->dev);
  (void)hipHostFree(se->host);
  ctx->session = nullptr;
  delete se;
  return st != AGILE_OK ? st : s2;
}

agile_status agile_serve(agile_ctx ctx, agile_store store, const agile_tables* tb, uint32_t K, uint32_t mode,
                         uint64_t nreq, const double* arrival_s, const int64_t* req_bag0, const int64_t* bag_off,
                         const int64_t* idx, float* out, double* latency_s, const agile_serve_opts* opts,
                         agile_serve_report* report) {
  agile_status s = check_usable(ctx);
  if (s) return s;
  if (!tb || !arrival_s || !req_bag0 || !bag_off || !out || !latency_s)
    return fail(ctx, AGILE_EINVAL, "serve: null pointer");
  if (nreq == 0) return AGILE_OK;
  for (uint64_t r = 0; r < nreq; ++r)
    if (req_bag0[r + 1] <= req_bag0[r] || (r && arrival_s[r] < arrival_s[r - 1]))
      return fail(ctx, AGILE_EINVAL, "serve: every request needs >= 1 bag; arrivals must not decrease");
  // the replay harness is one client of the session: it submits each request once it has
  // arrived and the session admits it, and collects outputs as they complete
  agile_session se = nullptr;
  if ((s = agile_session_open(ctx, store, tb, K, mode, opts, &se)) != AGILE_OK) return s;
  const uint32_t dim = tb->dim;
  uint64_t nlook = 0;
  std::vector<int64_t> rel;
  std::vector<uint64_t> ids(nreq, 0);
  std::vector<uint64_t> pending;  // submitted, not yet collected (request numbers)
  uint64_t next = 0, completed = 0, max_in = 0;
  const auto t0 = std::chrono::steady_clock::now();
  auto since = [&]() { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); };
  double last_progress = 0.0;
  const double limit_s = 4.0 * (double)ctx->cfg.timeout_ns * 1e-9 + 30.0;
  agile_status st_loop = AGILE_OK;
  while (completed < nreq) {
    const double now = since();
    bool moved = false;
    while (next < nreq && arrival_s[next] <= now) {
      const int64_t b0 = req_bag0[next], b1 = req_bag0[next + 1];
      rel.resize((size_t)(b1 - b0 + 1));
      for (int64_t b = b0; b <= b1; ++b) rel[b - b0] = bag_off[b] - bag_off[b0];
      const agile_status r = agile_session_submit(se, (uint32_t)(b1 - b0), rel.data(), idx + bag_off[b0], &ids[next]);
      if (r == AGILE_EAGAIN) break;  // no room yet: it waits, and so do the ones behind it
      if (r != AGILE_OK) {
        st_loop = r;
        break;
      }
      nlook += (uint64_t)(bag_off[b1] - bag_off[b0]);
      pending.push_back(next);
      max_in = std::max<uint64_t>(max_in, pending.size());
      ++next;
      moved = true;
    }
    if (st_loop != AGILE_OK) break;
    for (size_t i = 0; i < pending.size();) {
      const uint64_t q = pending[i];
      const agile_status r = agile_session_poll(se, ids[q], out + (uint64_t)req_bag0[q] * dim);
      if (r == AGILE_OK) {
        latency_s[q] = since() - arrival_s[q];
        pending[i] = pending.back();
        pending.pop_back();
        ++completed;
        moved = true;
      } else if (r == AGILE_EAGAIN) {
        ++i;
      } else {
        st_loop = r;
        break;
      }
    }
    if (st_loop != AGILE_OK) break;
    if (moved) {
      last_progress = now;
    } else if (now - last_progress > limit_s) {
      __atomic_store_n(ctx->abort_host, 1u, __ATOMIC_SEQ_CST);
      st_loop = fail(ctx, AGILE_ETIMEDOUT, "serve: no progress");
      break;
    }
  }
  const double elapsed = since();
  const uint64_t waves = se->user_waves;
  s = agile_session_close(se);
  if (st_loop != AGILE_OK) return st_loop;
  if (s != AGILE_OK) return s;
  if (report) {
    report->elapsed_s = elapsed;
    report->requests = nreq;
    report->bags = (uint64_t)req_bag0[nreq];
    report->lookups = nlook;
    report->max_inflight_requests = max_in;
    report->user_waves = waves;
  }
  return AGILE_OK;
}

// ---- diagnostics used by tests (declared in agile.h)
agile_status agile_debug_trace(agile_ctx ctx, agile_store store, const uint64_t* d_lines, const uint8_t* d_writes,
                               uint64_t n, uint8_t* d_hit, int32_t* d_way, void* stream) {
  agile_status s = check_usable(ctx);
  if (s) return s;
  if (store != ctx->store) return fail(ctx, AGILE_EINVAL, "trace: store is not open on this context");
  if (n == 0) return AGILE_OK;
  if (!d_lines || !d_hit || !d_way) return fail(ctx, AGILE_EINVAL, "trace: null pointer");
  launch_t li = make_launch(ctx, WPB, true);
  hipLaunchKernelGGL(k_trace, dim3(li.service_blocks + 1), dim3(WG), lds_of(ctx, (const void*)k_trace), (hipStream_t)stream, ctx->d, li, d_lines,
                     d_writes, n, d_hit, d_way);
  HIPCHK(ctx, hipGetLastError());
  return sync_stream(ctx, (hipStream_t)stream);
}

agile_status agile_debug_exclusive_scan_u64(const uint64_t* d_in, uint64_t* d_out, uint64_t n, void* stream) {
  if (n == 0) return AGILE_OK;
  if (!d_in || !d_out) return AGILE_EINVAL;
  hipStream_t hs = (hipStream_t)stream;
  void* work = nullptr;
  const size_t wb = 8 * sort::scan_work_elems(n) + 8;
  if (hipMalloc(&work, wb) != hipSuccess) {
    (void)hipGetLastError();
    return AGILE_ENOMEM;
  }
  bool ok = sort::exclusive_scan<uint64_t>(d_in, d_out, n, (uint64_t*)work, hs);
  ok = hipStreamSynchronize(hs) == hipSuccess && ok;
  (void)hipFree(work);
  return ok ? AGILE_OK : AGILE_EHIP;
}

agile_status agile_debug_radix_sort_u64(uint64_t* d_keys, uint64_t n, uint32_t lo, uint32_t hi, void* stream) {
  if (n == 0) return AGILE_OK;
  if (!d_keys || lo > hi || hi > 64) return AGILE_EINVAL;
  hipStream_t hs = (hipStream_t)stream;
  void* work = nullptr;
  if (hipMalloc(&work, sort::radix_work_bytes(n)) != hipSuccess) {
    (void)hipGetLastError();
    return AGILE_ENOMEM;
  }
  uint64_t* sorted = nullptr;
  bool ok = sort::radix_sort(d_keys, n, lo, hi, work, hs, &sorted);
  if (ok && sorted != d_keys)
    ok = hipMemcpyAsync(d_keys, sorted, n * 8, hipMemcpyDeviceToDevice, hs) == hipSuccess;
  ok = hipStreamSynchronize(hs) == hipSuccess && ok;
  (void)hipFree(work);
  return ok ? AGILE_OK : AGILE_EHIP;
}

agile_status agile_debug_counters(agile_ctx ctx, uint64_t* out, uint32_t n) {
  if (!ctx || !out) return AGILE_EINVAL;
  std::vector<uint64_t> c((size_t)C_COUNT * CSTRIDE);
  HIPCHK(ctx, hipDeviceSynchronize());
  HIPCHK(ctx, hipMemcpy(c.data(), ctx->d.cnt, c.size() * 8, hipMemcpyDeviceToHost));
  for (uint32_t i = 0; i < n; ++i) out[i] = i < C_COUNT ? c[(size_t)i * CSTRIDE] : 0;
  return AGILE_OK;
}

agile_status agile_debug_dump(agile_ctx ctx, int64_t* d_tags, uint8_t* d_states, uint32_t* d_rc, void* stream) {
  if (!ctx || !d_tags || !d_states || !d_rc) return AGILE_EINVAL;
  const uint32_t nb = (ctx->d.num_lines + 255) / 256;
  hipLaunchKernelGGL(k_dump, dim3(nb), dim3(256), 0, (hipStream_t)stream, ctx->d, d_tags, d_states, d_rc);
  HIPCHK(ctx, hipGetLastError());
  HIPCHK(ctx, hipStreamSynchronize((hipStream_t)stream));
  return AGILE_OK;
}

}  // extern "C"
