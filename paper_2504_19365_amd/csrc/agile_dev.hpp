// agile_dev.hpp - device side of the block-I/O path for gfx950 (wave64, 8 XCDs).
//
// Contents, bottom-up:
//   * memory-model helpers (agent scope = every XCD of the device),
//   * wavefront helpers (ballot / mbcnt / readlane),
//   * NVMe-style queue pair: 64-byte SQE, 16-byte CQE, lap-tagged slot states,
//   * wavefront-aggregated submission with the doorbell serialisation of Alg. 2,
//   * the emulated NVMe controller (service wavefronts, latency + IOPS cap),
//   * the completion service (Alg. 1, one 64-entry window per wavefront),
//   * the cache line state machine of Sec. 3.4 with clock replacement,
//   * the wavefront-level "request chunk" API used by every workload kernel.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ag {

// ------------------------------------------------------------------ memory model
template <class T>
__device__ __forceinline__ T ld_acq(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ T ld_rlx(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T, class U>
__device__ __forceinline__ void st_rel(T* p, U v) {
  __hip_atomic_store(p, (T)v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T, class U>
__device__ __forceinline__ void st_rlx(T* p, U v) {
  __hip_atomic_store(p, (T)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T, class U>
__device__ __forceinline__ T add_rlx(T* p, U v) {
  return __hip_atomic_fetch_add(p, (T)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T, class U>
__device__ __forceinline__ T add_acqrel(T* p, U v) {
  return __hip_atomic_fetch_add(p, (T)v, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T, class U>
__device__ __forceinline__ T add_rel(T* p, U v) {
  return __hip_atomic_fetch_add(p, (T)v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T, class U>
__device__ __forceinline__ bool cas(T* p, T& expected, U desired) {
  return __hip_atomic_compare_exchange_strong(p, &expected, (T)desired, __ATOMIC_ACQ_REL,
                                              __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T, class U>
__device__ __forceinline__ T and_rlx(T* p, U v) {
  return __hip_atomic_fetch_and(p, (T)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T, class U>
__device__ __forceinline__ T or_rlx(T* p, U v) {
  return __hip_atomic_fetch_or(p, (T)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void fence_acq() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }
__device__ __forceinline__ void fence_rel() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
__device__ __forceinline__ void fence_rel_sys() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, ""); }
__device__ __forceinline__ void fence_acq_sys() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, ""); }
// Completes this wave's outstanding loads before a following relaxed atomic; enough to
// retire read-only pins (no stores need publishing).
__device__ __forceinline__ void loads_done() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
}

__device__ __forceinline__ uint64_t now() { return __builtin_amdgcn_s_memrealtime(); }

// ------------------------------------------------------------------ wave64 helpers
__device__ __forceinline__ uint32_t lane() { return __lane_id(); }
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }
__device__ __forceinline__ uint32_t mbcnt(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
__device__ __forceinline__ uint32_t rdlane(uint32_t v, uint32_t l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)l);
}
__device__ __forceinline__ uint64_t rdlane64(uint64_t v, uint32_t l) {
  return ((uint64_t)rdlane((uint32_t)(v >> 32), l) << 32) | rdlane((uint32_t)v, l);
}
// Makes a value wave-uniform (every lane takes the first active lane's value).
__device__ __forceinline__ uint32_t uni(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}
__device__ __forceinline__ uint64_t uni64(uint64_t v) {
  return ((uint64_t)uni((uint32_t)(v >> 32)) << 32) | uni((uint32_t)v);
}
__device__ __forceinline__ uint32_t ffs64(uint64_t m) { return (uint32_t)__builtin_ctzll(m); }
__device__ __forceinline__ uint32_t shfl32(uint32_t v, uint32_t src) {
  return (uint32_t)__shfl((int)v, (int)src, 64);
}

// ------------------------------------------------------------------ shared layouts
// Cache line metadata word:
//   bits 0-2 state, bit 3 clock reference bit, bits 4-23 pin count,
//   bits 24-31 generation (bumped on every refill), bits 32-63 tag (line id in store).
enum : uint32_t { ST_INVALID = 0, ST_FETCHING = 1, ST_READY = 2, ST_DIRTY = 3, ST_WRITEBACK = 4 };
constexpr uint64_t M_STATE = 7ull, M_REF = 8ull, RC_ONE = 1ull << 4, RC_MASK = 0xFFFFFull << 4;
constexpr uint32_t GEN_SHIFT = 24, TAG_SHIFT = 32;
// Pins a line may hold.  Pins are taken with one atomic add and given back when the
// line turns out not to be the one wanted or to be at the limit, so the 20-bit count
// must also hold every addition in flight above the limit: at most 64 per wavefront
// (8,192 wavefronts on 256 CUs), 2^19 in all, and 2^18 + 2^19 < 2^20.
constexpr uint32_t RC_LIMIT = 1u << 18;
static_assert(RC_LIMIT + 64u * 8192u < (1u << 20), "the pin count could carry into the generation");
__device__ __forceinline__ uint32_t m_state(uint64_t m) { return (uint32_t)(m & M_STATE); }
__device__ __forceinline__ uint32_t m_rc(uint64_t m) { return (uint32_t)((m & RC_MASK) >> 4); }
__device__ __forceinline__ uint32_t m_gen(uint64_t m) { return (uint32_t)(m >> GEN_SHIFT) & 0xFF; }
__device__ __forceinline__ uint32_t m_tag(uint64_t m) { return (uint32_t)(m >> TAG_SHIFT); }
__device__ __forceinline__ bool m_valid_data(uint32_t st) {
  return st == ST_READY || st == ST_DIRTY || st == ST_WRITEBACK;
}

// Slot state word of an SQ entry: (ticket << 2) | state, modulo 2^32.  The ticket is the
// lap-unique sequence number of the command that owns (or may next own) the slot.
enum : uint32_t { SLOT_EMPTY = 0, SLOT_UPDATED = 1, SLOT_ISSUED = 2 };

// NVM command set opcodes.
enum : uint32_t { OPC_WRITE = 0x01, OPC_READ = 0x02 };

// 64-byte submission entry with the field positions of an NVMe command: CDW0 holds the
// opcode and the command identifier (CID = slot index), PRP1 the HBM line address,
// CDW10-11 the starting block (SLBA), CDW12 bits 0-15 the block count minus one.  CDW2
// (reserved in NVMe) carries the cache line index so the completion can find it.
struct alignas(64) sqe_t {
  uint32_t cdw0, nsid, cdw2, cdw3;
  uint64_t mptr, prp1, prp2, slba;
  uint32_t cdw12, cdw13, cdw14, cdw15;
};
// 16-byte completion entry: DW0 command specific (the cache line index), DW1 the opcode,
// DW2 SQ head | SQ id << 16, DW3 CID | phase << 16 | status << 17.
struct alignas(16) cqe_t {
  uint32_t dw0, dw1, dw2, dw3;
};

// Per queue pair control words, one 128-byte segment per writer group.
struct alignas(128) qp_t {
  uint32_t ticket;            // submitters: next reservation
  uint32_t _p0[31];
  uint32_t db;                // SQ tail doorbell (written under db_lock)
  uint32_t db_lock;
  uint32_t _p1[30];
  uint32_t fetch;             // controller: next SQE to fetch
  uint32_t cq_tail;           // controller: next CQ slot to post
  uint32_t _p2[30];
  uint32_t cq_head;           // completion service: CQ head doorbell (window start)
  uint32_t cq_mask_lo, cq_mask_hi;  // completion service: window mask kept between launches
  uint32_t _p3[29];
};

// Counters, one 128-byte segment each.
enum : uint32_t {
  C_SUBMITTED = 0, C_COMPLETED, C_USER_DONE, C_WORK, C_REQUESTS, C_HITS, C_MISSES, C_READS,
  C_WRITES, C_WB_EVICT, C_WB_FLUSH, C_EAGAIN, C_SQ_SPINS, C_CTRL_CMDS, C_CQ_ENTRIES, C_AUX0,
  C_AUX1, C_SVC_START, C_CTRL_FETCH, C_CTRL_LOOPS, C_CQ_LOOPS, C_WROWS,
  // stage timers (ticks of s_memrealtime, summed over wavefronts; profile flag only)
  P_CTRL_FETCH, P_CTRL_COPY, P_CTRL_POST, P_CTRL_HOLD, P_CTRL_IDLE, P_CTRL_NOROOM, P_CQ_BUSY,
  P_CQ_IDLE, P_U_ISSUE, P_U_SUBMIT, P_U_WAIT, P_U_CONSUME, P_TOK_LEAD, P_TOK_N, P_U_DESC,
  P_U_LIFE, C_SVC_EXIT, C_IMG_EPOCH,
  // work counters of partitions 1..7 (partition 0 is C_WORK)
  C_WORK_P1, C_WORK_P2, C_WORK_P3, C_WORK_P4, C_WORK_P5, C_WORK_P6, C_WORK_P7,
  // resident-hit pass: bags it deferred to the I/O pass
  C_DEFER,
  // entries of the pending lists taken by the launch
  C_PEND,
  // lookups of a launch whose bags went through the resident-hit pass, and of the bags
  // it deferred: the pass's own requests and hits are their difference (it counts
  // nothing itself; agile_get_stats adds the difference)
  C_HIT_TOTAL, C_DEFLEN, C_COUNT
};
constexpr uint32_t CSTRIDE = 16;  // u64 per counter

// Device error codes (mapped to agile_status on the host).
enum : uint32_t { E_NONE = 0, E_TIMEDOUT = 1, E_IO = 2, E_PROTO = 3, E_STATE = 4 };

struct dev_ctx {
  // cache
  uint8_t* lines;
  uint64_t* meta;
  uint32_t* hand;
  uint32_t* set_lock;
  uint32_t num_lines, num_sets, assoc, line_shift;
  uint32_t sets_pow2, blocks_per_line;
  // queues
  sqe_t* sq;
  cqe_t* cq;
  uint32_t* slot;
  qp_t* qp;
  uint32_t num_qp, depth, depth_shift, _q0;
  // store (4 KiB blocks), striped over n_dev emulated devices one cache line at a time
  // (Sec. 4.3's interleaving, request i to device i mod n): line l lives on device
  // l mod n_dev as that device's line l / n_dev.  Queue pair q belongs to device
  // q mod n_dev, and so does its token bucket.
  uint8_t* image;               // device 0's image (the only one when n_dev == 1)
  const uint64_t* dev_image;    // [n_dev] base address of each device's image
  uint64_t store_blocks;        // blocks of the whole (logical) store
  uint64_t dev_blocks;          // blocks of each device
  uint32_t n_dev, _s0;
  // emulator
  uint64_t lat_ticks;
  uint64_t tok_fp;  // ticks per command in TOK_FRAC-bit fixed point; 0 = no cap
  uint64_t tok_max; // largest lead a reservation can legitimately have (same units)
  uint64_t* next_tok;
  // control
  uint64_t* cnt;
  uint32_t* err;
  uint32_t* abort_flag;  // pinned host word: the host watchdog raises it
  uint32_t* abort_dev;   // device word that every wait polls
  uint64_t* err_info;
  uint64_t timeout_ticks;
  uint32_t flags;
  uint32_t _c0;
  // lock-chain debugging (flag FLAG_LOCKCHAIN): what each spinning wave waits for, and
  // the chain the first timed-out wave recorded
  uint64_t* waits;  // [2 * WAIT_SLOTS]: per wave number, what it waits for and when it last looked
  uint64_t* chain;  // [1 + 3 * LC_MAX]
  // reads into user buffers (Sec. 3.4.1): each cache line's list of buffers waiting for
  // its fill, the list entries of a launch, and the Share Table (block -> buffer)
  uint32_t* pend_head;   // [num_lines]: first entry, PEND_EMPTY, or PEND_CLOSED once drained
  uint64_t* pend;        // [2 * PEND_CAP]: destination address; next entry | block offset << 32
  uint64_t* share_key;   // [SHARE_CAP]: block + 1, 0 = free
  uint64_t* share_buf;   // [SHARE_CAP]: the owner's buffer
  uint32_t* share_refs;  // [SHARE_CAP]: holders (owner + sharers); SHARE_BUSY while installing
};
constexpr uint32_t PEND_EMPTY = 0xFFFFFFFFu, PEND_CLOSED = 0xFFFFFFFEu;
constexpr uint32_t PEND_CAP = 1u << 20;
constexpr uint32_t SHARE_CAP = 1u << 18, SHARE_PROBES = 64, SHARE_BUSY = 0xFFFFFFFFu;

struct launch_t {
  uint32_t service_blocks;  // leading workgroups that run service wavefronts
  uint32_t n_ctrl, n_cq;    // controller / completion wavefronts
  uint32_t user_waves;      // user wavefronts in this launch (the service waits for all)
  uint32_t prio;            // raise service issue priority
  uint32_t _l0;
};

// Threads per workgroup: 16 wavefronts.  Kernels that carry service wavefronts also
// reserve more than half of a CU's LDS, so that exactly one workgroup fits per CU: the
// leading service workgroups then own whole CUs and no user wave shares a SIMD or a
// memory pipeline with the emulated controller or the completion service.
constexpr uint32_t WG = 1024;
constexpr uint32_t FLAG_PROFILE = 0x4;
constexpr uint32_t FLAG_LOCKCHAIN = 0x8;
constexpr uint32_t WAIT_SLOTS = 1u << 16;
constexpr uint32_t LC_MAX = 16;
// What a spinning wave waits for (error reports and lock-chain debugging): the kind in
// the top byte, the object below it.
enum : uint32_t {
  W_SQ_SLOT = 0x01,  // a free slot of SQ q for ticket t: (q << 32) | t
  W_SETLOCK = 0x0A,  // the lock of the set of store line id
  W_WB = 0x0B,       // its own write-back of cache line index
  W_FILL = 0x0D,     // the fill of cache line index
  W_TICKET = 0x0E,   // a ticket's line (cache line index)
  W_WAY = 0x0F,      // an evictable way (after EAGAIN)
  W_CLAIM = 0x10,    // a write claim of cache line index
  W_BACKLOG = 0x11   // the store's backlog to shrink below `id` commands (prefetch)
};
__host__ __device__ constexpr uint64_t wi(uint32_t kind, uint64_t id) {
  return ((uint64_t)kind << 56) | (id & ((1ull << 56) - 1));
}
// Token times of the IOPS cap are kept in 44.20 fixed point of the wall clock, modulo
// 2^64: the integer part wraps after about two days of 100 MHz ticks, so a stored token
// time is only used through its difference to now, and only while that lead is positive
// and no larger than the queues can account for (an idle or never-used bucket can sit at
// any distance, with either sign).
constexpr uint32_t TOK_FRAC = 20;
constexpr uint32_t WPB = WG / 64;
// Workgroups are dealt to the 8 XCDs round robin, and each XCD has its own L2 and its
// own share of the fabric path to host memory.  Service roles are numbered across the
// service workgroups first (role = wave * service_blocks + workgroup) and there are at
// least this many service workgroups, so the controller wavefronts, which do all the
// PCIe copying, are spread over every XCD.
constexpr uint32_t XCDS = 8;
__host__ __device__ constexpr uint32_t service_blocks_for(uint32_t service_waves) {
  const uint32_t packed = (service_waves + WPB - 1) / WPB;               // WPB roles per group
  const uint32_t spread = service_waves < XCDS ? service_waves : XCDS;  // one group per XCD
  return packed > spread ? packed : spread;
}
static_assert(service_blocks_for(80) == 8 && service_blocks_for(144) == 9 && service_blocks_for(2) == 2 &&
                  service_blocks_for(1) == 1,
              "service workgroups: at least one per XCD, at most WPB roles each");

// Dynamic work is split over WORK_PARTS counters, each in its own 128-byte segment, so
// that thousands of waves taking work do not all meet at one address.
constexpr uint32_t WORK_PARTS = 8;
__device__ __forceinline__ uint32_t work_counter(uint32_t p) { return p == 0 ? C_WORK : C_WORK_P1 + (p - 1); }

__device__ __forceinline__ uint64_t* counter(const dev_ctx& c, uint32_t i) {
  return c.cnt + (size_t)i * CSTRIDE;
}
__device__ __forceinline__ void count(const dev_ctx& c, uint32_t i, uint64_t v) {
  if (v) add_rlx(counter(c, i), v);
}
__device__ __forceinline__ bool profiling(const dev_ctx& c) { return (c.flags & FLAG_PROFILE) != 0; }
__device__ __forceinline__ bool lockchain(const dev_ctx& c) { return (c.flags & FLAG_LOCKCHAIN) != 0; }
// The wave's number in its launch.
__device__ __forceinline__ uint32_t wave_gid() { return (blockIdx.x * blockDim.x + threadIdx.x) >> 6; }
// Adds now() - t to timer i (lane 0 only, profile flag only); returns now().
__device__ __forceinline__ uint64_t ptick(const dev_ctx& c, uint32_t i, uint64_t t) {
  if (!profiling(c)) return 0;
  const uint64_t n = now();
  if (lane() == 0) add_rlx(c.cnt + (size_t)i * CSTRIDE, n - t);
  return n;
}
// Abort has two words.  The host watchdog can only raise the one in pinned host memory;
// waits poll the device word, since thousands of waves reading host memory in their
// spin loops would flood the PCIe link that the controller's copies use.  A few waves
// (one controller wavefront, the serving mirror, and every spinning wave at a low rate)
// look at the host word and copy a raised flag into the device word.
__device__ __forceinline__ bool aborted(const dev_ctx& c) { return uni(ld_rlx(c.abort_dev)) != 0; }
__device__ __forceinline__ bool host_abort_poll(const dev_ctx& c) {
  if (!uni(__hip_atomic_load(c.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM))) return false;
  if (lane() == 0) st_rlx(c.abort_dev, 1u);
  return true;
}
// Kept out of line (a cold path) with plain pointer arguments: a reference to the whole
// context would force the kernel to keep a copy of it in scratch memory.
__device__ __noinline__ void raise_error_at(uint32_t* err, uint64_t* err_info, uint32_t* abort_dev,
                                            uint32_t* abort_flag, uint32_t code, uint64_t info) {
  uint32_t z = 0;
  if (cas(err, z, code)) st_rlx(err_info, info);
  st_rlx(abort_dev, 1u);
  __hip_atomic_store(abort_flag, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void raise_error(const dev_ctx& c, uint32_t code, uint64_t info) {
  raise_error_at(c.err, c.err_info, c.abort_dev, c.abort_flag, code, info);
}

// Bounded spin helper: returns false (and raises E_TIMEDOUT) when the deadline passes or
// the context is aborted.
// Backoff: about 0.1 us doubling to about 3 us for the first few polls, then a sleep of
// about an eighth of the time already waited (at most about 50 us), so a wave is never
// woken more than ~12% late and thousands of waves that wait for queued I/O (milliseconds
// when the device is saturated) do not flood the memory system that the controller's
// copies share.
__device__ void lc_walk(const dev_ctx& c, uint32_t w0, uint64_t what);
// Lock-chain mode: a spinning wave notes what it waits for when it starts and the time
// at every step, so a record whose time is older than LC_FRESH ticks (far more than the
// longest back-off between steps) belongs to a wave that has stopped waiting.
constexpr uint64_t LC_FRESH = 20000;  // 200 us
__device__ __forceinline__ void lc_note(const dev_ctx& c, uint64_t info, bool first) {
  const uint32_t w = wave_gid();
  if (w < WAIT_SLOTS && lane() == ffs64(ballot(true))) {
    if (first) st_rlx(c.waits + 2 * w, info);
    st_rlx(c.waits + 2 * w + 1, now());
  }
}
struct spin_t {
  uint64_t t0;
  uint32_t n;
  __device__ spin_t() : t0(now()), n(0) {}
  __device__ __forceinline__ bool step(const dev_ctx& c, uint64_t info) {
    ++n;
    if (lockchain(c)) lc_note(c, info, n == 1);
    if (n < 7) {
      const uint32_t reps = 1u << (n - 1);
      for (uint32_t r = 0; r < reps; ++r) __builtin_amdgcn_s_sleep(4);
    } else {
      // s_sleep(127) is 127 * 64 clocks, about 340 wall-clock ticks (10 ns each)
      const uint64_t k = (now() - t0) / (8 * 340);
      const uint32_t reps = k < 1 ? 1u : (k > 14 ? 14u : (uint32_t)k);
      for (uint32_t r = 0; r < reps; ++r) __builtin_amdgcn_s_sleep(127);
    }
    if (n >= 7 || (n & 3) == 0) {
      if (aborted(c)) return false;
      if ((n & 63) == 0 && host_abort_poll(c)) return false;  // every few ms
      if (now() - t0 > c.timeout_ticks) {
        if (lane() == ffs64(ballot(true))) {
          if (lockchain(c)) lc_walk(c, wave_gid(), info);
          raise_error(c, E_TIMEDOUT, info);
        }
        return false;
      }
    }
    return true;
  }
};

__device__ __forceinline__ uint32_t set_of(const dev_ctx& c, uint32_t line_id) {
  return c.sets_pow2 ? (line_id & (c.num_sets - 1)) : (line_id % c.num_sets);
}
__device__ __forceinline__ uint8_t* line_ptr(const dev_ctx& c, uint32_t idx) {
  return c.lines + ((uint64_t)idx << c.line_shift);
}

// ------------------------------------------------------------------ submission (Alg. 2)
// Wavefront-aggregated: the lanes with `want` reserve consecutive tickets of SQ `q` with
// one atomic, then every lane waits until its slot's previous lap is EMPTY, writes its
// 64-byte command and marks the slot UPDATED.  While any of its commands is unissued the
// wave also tries the doorbell lock; the holder scans forward 64 slots at a time,
// turning UPDATED slots of the expected lap into ISSUED until the first slot that is not
// (an unwritten or empty entry), then stores the new tail into the doorbell.  The wave
// returns once its last ticket is behind the doorbell.  Returns false on abort/timeout.
__device__ __forceinline__ bool submit(const dev_ctx& c, uint32_t q, bool want, uint32_t opc, uint32_t line_idx,
                       uint64_t slba, uint32_t nblk) {
  const uint64_t m = ballot(want);
  if (!m) return true;
  const uint32_t n = __popcll(m);
  const uint32_t rank = mbcnt(m);
  qp_t* qs = c.qp + q;
  uint32_t base = 0;
  if (lane() == ffs64(m)) {
    base = add_rlx(&qs->ticket, n);
    add_rlx(counter(c, C_SUBMITTED), (uint64_t)n);
    add_rlx(counter(c, opc == OPC_READ ? C_READS : C_WRITES), (uint64_t)n);
  }
  base = rdlane(base, ffs64(m));
  const uint32_t T = base + rank;
  const uint32_t dmask = c.depth - 1;
  const uint32_t s = T & dmask;
  uint32_t* slots = c.slot + (size_t)q * c.depth;
  bool written = !want;
  spin_t sp;
  uint32_t spins = 0;
  for (;;) {
    bool progress = false;
    if (!written) {
      if (ld_rlx(slots + s) == ((T << 2) | SLOT_EMPTY)) {
        sqe_t* e = c.sq + (size_t)q * c.depth + s;
        uint4* w = reinterpret_cast<uint4*>(e);
        const uint64_t prp1 = (uint64_t)(uintptr_t)line_ptr(c, line_idx);
        w[0] = make_uint4(opc | (s << 16), 1u, line_idx, T);
        w[1] = make_uint4(0u, 0u, (uint32_t)prp1, (uint32_t)(prp1 >> 32));
        w[2] = make_uint4(0u, 0u, (uint32_t)slba, (uint32_t)(slba >> 32));
        w[3] = make_uint4(nblk - 1, 0u, 0u, 0u);
        st_rel(slots + s, (T << 2) | SLOT_UPDATED);
        written = true;
        progress = true;
      }
    }
    progress = ballot(progress) != 0;
    const uint32_t db = uni(ld_rlx(&qs->db));
    if ((int32_t)(db - (base + n)) >= 0) break;  // every command of this wave is issued
    if (ballot(written && want)) {
      uint32_t got = 0;
      if (lane() == 0) {
        uint32_t z = 0;
        got = cas(&qs->db_lock, z, 1u) ? 1u : 0u;
      }
      got = rdlane(got, 0);
      if (got) {
        uint32_t p = ld_rlx(&qs->db);
        const uint32_t p0 = p;
        for (;;) {
          const uint32_t t = p + lane();
          const bool upd = ld_rlx(slots + (t & dmask)) == ((t << 2) | SLOT_UPDATED);
          const uint64_t b = ballot(upd);
          const uint32_t k = (~b == 0ull) ? 64u : ffs64(~b);
          if (lane() < k) st_rlx(slots + (t & dmask), (t << 2) | SLOT_ISSUED);
          p += k;
          if (k < 64) break;
        }
        // one acquire for the scanned entries, one release for the doorbell and the lock
        fence_acq();
        fence_rel();
        if (lane() == 0) {
          if (p != p0) st_rlx(&qs->db, p);  // the doorbell write
          st_rlx(&qs->db_lock, 0u);
        }
        if (p != p0) progress = true;
      }
    }
    if (!progress) {
      ++spins;
      if (!sp.step(c, wi(W_SQ_SLOT, ((uint64_t)q << 32) | T))) return false;
    }
  }
  if (spins && lane() == 0) count(c, C_SQ_SPINS, spins);
  return true;
}

// Submits one command per lane with `want` for a whole cache line of the store (a
// line at a device's end may be short), each to the queue pair of the line's device in
// the wave's group of queue pairs ((q / n_dev) * n_dev + device): one wave-wide
// submission per device present among the lanes.
__device__ __forceinline__ bool submit_line(const dev_ctx& c, uint32_t q, bool want, uint32_t opc,
                                            uint32_t line_idx, uint32_t line_id) {
  uint64_t todo = ballot(want);
  if (!todo) return true;
  const bool one = c.n_dev == 1;
  const uint32_t d = one ? 0u : line_id % c.n_dev;
  const uint32_t bpl = c.blocks_per_line;
  const uint64_t slba = (uint64_t)(one ? line_id : line_id / c.n_dev) * bpl;
  uint32_t nblk = bpl;
  if (want && slba + nblk > c.dev_blocks) nblk = (uint32_t)(c.dev_blocks - slba);
  const uint32_t qg = one ? q : q - q % c.n_dev;
  do {
    const uint32_t dd = rdlane(d, ffs64(todo));
    const bool mine = want && d == dd;
    if (!submit(c, qg + dd, mine, opc, line_idx, slba, nblk)) return false;
    todo &= ~ballot(mine);
  } while (todo);
  return true;
}

// ------------------------------------------------------------------ service wavefronts
__device__ __forceinline__ bool service_should_exit(const dev_ctx& c, const launch_t& li) {
  if (aborted(c)) return true;
  if (uni64(ld_rlx(counter(c, C_USER_DONE))) < li.user_waves) return false;
  const uint64_t sub = uni64(ld_rlx(counter(c, C_SUBMITTED)));
  const uint64_t com = uni64(ld_rlx(counter(c, C_COMPLETED)));
  return com == sub;
}

// Position of the r-th (0-based) set bit of m; r < popcount(m).
__device__ __forceinline__ uint32_t nth_set_bit(uint64_t m, uint32_t r) {
  uint32_t pos = 0;
#pragma unroll
  for (uint32_t step = 32; step; step >>= 1)
    if ((uint32_t)__popcll(m & ((1ull << (pos + step)) - 1ull)) <= r) pos += step;
  return pos;
}
__device__ __forceinline__ uint64_t shfl64(uint64_t v, uint32_t src) {
  return ((uint64_t)shfl32((uint32_t)(v >> 32), src) << 32) | shfl32((uint32_t)v, src);
}

// Copies one 4 KiB block with the whole wave: 16-byte lanes, 1 KiB per instruction, so
// that each instruction touches a single page of the pinned image.  `nb` (1..4) blocks
// are copied together with all their loads issued before the stores.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) u32x4 gmem_u32x4;

// Copies NB 4 KiB blocks with one wavefront: every lane moves 16 bytes of each quarter of
// each block, all NB * 4 loads in flight before the first store (PCIe reads are latency-
// bound, so bytes in flight per wave set the copy rate).
template <uint32_t NB>
__device__ __forceinline__ void copy_n(uint8_t* const (&dst)[4], const uint8_t* const (&src)[4]) {
  u32x4 v[NB][4];
#pragma unroll
  for (uint32_t b = 0; b < NB; ++b) {
    const gmem_u32x4* s = (const gmem_u32x4*)src[b];
#pragma unroll
    for (uint32_t i = 0; i < 4; ++i) v[b][i] = s[i * 64 + lane()];
  }
#pragma unroll
  for (uint32_t b = 0; b < NB; ++b) {
    gmem_u32x4* d = (gmem_u32x4*)dst[b];
#pragma unroll
    for (uint32_t i = 0; i < 4; ++i) d[i * 64 + lane()] = v[b][i];
  }
}
__device__ __forceinline__ void copy_blocks(uint8_t* const (&dst)[4], const uint8_t* const (&src)[4], uint32_t nb) {
  switch (nb) {
    case 1: copy_n<1>(dst, src); break;
    case 2: copy_n<2>(dst, src); break;
    case 3: copy_n<3>(dst, src); break;
    default: copy_n<4>(dst, src); break;
  }
}
__device__ __forceinline__ void copy_cmds(const dev_ctx& c, uint64_t ready, uint32_t p_opc, uint32_t p_nblk,
                          uint32_t p_status, uint64_t p_slba, uint64_t p_prp, uint32_t p_q) {
  // the block pointers are written at constant indices only, so they stay in registers
  uint8_t* dst[4] = {nullptr, nullptr, nullptr, nullptr};
  const uint8_t* src[4] = {nullptr, nullptr, nullptr, nullptr};
  uint32_t k = 0;
  for (uint64_t rem = ready; rem; rem &= rem - 1) {
    const uint32_t l = ffs64(rem);
    if (rdlane(p_status, l)) continue;
    const uint32_t nblk = rdlane(p_nblk, l);
    const bool rd = rdlane(p_opc, l) == OPC_READ;
    uint8_t* hbm = (uint8_t*)(uintptr_t)rdlane64(p_prp, l);
    uint8_t* base = c.image;
    if (c.n_dev > 1) base = (uint8_t*)(uintptr_t)c.dev_image[rdlane(p_q, l) % c.n_dev];
    uint8_t* img = base + (rdlane64(p_slba, l) << 12);
    for (uint32_t b = 0; b < nblk; ++b) {
      const uint64_t o = (uint64_t)b << 12;
#pragma unroll
      for (uint32_t i = 0; i < 4; ++i)
        if (i == k) {
          src[i] = rd ? img + o : hbm + o;
          dst[i] = rd ? hbm + o : img + o;
        }
      if (++k == 4) {
        copy_blocks(dst, src, 4);
        k = 0;
      }
    }
  }
  if (k) copy_blocks(dst, src, k);
}

// Emulated NVMe controller wavefront (Sec. 2.1 device side).  It keeps up to 64 commands
// in flight, one per lane: it fetches new entries from its queue pairs once their doorbell
// moves, stamps the fetch time with s_memrealtime, takes a token from the store's global
// bucket when an IOPS cap is set, and completes a command once
// now >= max(fetch + latency, token time): the block(s) are copied across PCIe between
// the pinned image and the HBM line, then a phase-tagged CQE is posted.
__device__ __forceinline__ void controller(const dev_ctx& c, const launch_t& li, uint32_t cw) {
  const uint32_t dmask = c.depth - 1;
  const bool shared = li.n_ctrl > c.num_qp;
  const uint32_t qstep = li.n_ctrl < c.num_qp ? li.n_ctrl : c.num_qp;
  const uint32_t q0 = cw % c.num_qp;
  // per-lane pending command
  bool pend = false, p_copied = false;
  uint32_t p_q = 0, p_opc = 0, p_cid = 0, p_line = 0, p_nblk = 0, p_status = 0;
  uint64_t p_slba = 0, p_prp = 0, p_deadline = 0;
  uint64_t idle_since = now();
  uint64_t busy = 0;
  uint32_t loops = 0, idle_rounds = 0;
  uint64_t host_seen = idle_since;
  uint64_t img_epoch = ~0ull;  // unknown: the first copy of the launch drops stale lines
  for (;;) {
    if (((++loops) & 1023) == 0 && lane() == 0) count(c, C_CTRL_LOOPS, 1);
    const uint64_t t = now();
    if (cw == 0 && t - host_seen > 2000) {  // mirror the host's abort flag every 20 us
      host_seen = t;
      if (host_abort_poll(c)) break;
    }
    uint64_t tp = t;
    bool progress = false;
    // 1. fetch into free lanes
    uint64_t freem = ballot(!pend);
    for (uint32_t q = q0; q < c.num_qp && freem; q += qstep) {
      qp_t* qs = c.qp + q;
      // the fetch pointer first: a doorbell read before it may be older than a fetch
      // pointer that other controllers have since advanced, and the difference would wrap
      const uint32_t f = uni(ld_acq(&qs->fetch));
      const uint32_t db = uni(ld_rlx(&qs->db));
      uint32_t avail = db - f;
      if (avail == 0 || avail > c.depth) continue;
      fence_acq();  // the entries behind the doorbell are visible from here on
      const uint32_t nfree = __popcll(freem);
      const uint32_t k = avail < nfree ? avail : nfree;
      if (shared) {
        uint32_t ok = 0;
        if (lane() == 0) {
          uint32_t e = f;
          ok = cas(&qs->fetch, e, f + k) ? 1u : 0u;
        }
        if (!rdlane(ok, 0)) continue;
      } else if (lane() == 0) {
        st_rlx(&qs->fetch, f + k);
      }
      if (lane() == 0) count(c, C_CTRL_FETCH, k);
      const uint32_t r = mbcnt(freem);
      const bool take = ((freem >> lane()) & 1ull) && r < k;
      // token bucket for the IOPS cap: reserve k consecutive release times; tok0 is the
      // first one, relative to t
      uint64_t tok0 = 0;
      if (c.tok_fp) {
        uint64_t* bucket = c.next_tok + (size_t)(q % c.n_dev) * 16;  // the device's own
        if (lane() == 0) {
          const uint64_t tn = t << TOK_FRAC;  // wraps; only differences are used
          uint64_t old = ld_rlx(bucket);
          for (;;) {
            // a lead beyond what every queued command could account for is a bucket
            // that went idle (or was never used): it restarts at now
            const uint64_t lead = old - tn;
            const uint64_t first = ((int64_t)lead > 0 && lead <= c.tok_max) ? old : tn;
            if (cas(bucket, old, first + (uint64_t)k * c.tok_fp)) {
              tok0 = first - tn;
              if (profiling(c)) {
                count(c, P_TOK_LEAD, tok0 >> TOK_FRAC);
                count(c, P_TOK_N, 1);
              }
              break;
            }
          }
        }
        tok0 = rdlane64(tok0, 0);
      }
      if (take) {
        const uint32_t s = (f + r) & dmask;
        const sqe_t* e = c.sq + (size_t)q * c.depth + s;
        const uint4 w0 = reinterpret_cast<const uint4*>(e)[0];
        const uint4 w1 = reinterpret_cast<const uint4*>(e)[1];
        const uint4 w2 = reinterpret_cast<const uint4*>(e)[2];
        const uint4 w3 = reinterpret_cast<const uint4*>(e)[3];
        p_q = q;
        p_opc = w0.x & 0xFF;
        p_cid = w0.x >> 16;
        p_line = w0.z;
        p_prp = ((uint64_t)w1.w << 32) | w1.z;
        p_slba = ((uint64_t)w2.w << 32) | w2.z;
        p_nblk = (w3.x & 0xFFFF) + 1;
        p_status = 0;
        const uint64_t lo = (uint64_t)(uintptr_t)c.lines;
        const uint64_t hi = lo + ((uint64_t)c.num_lines << c.line_shift);
        if (p_cid != s || (p_opc != OPC_READ && p_opc != OPC_WRITE) || w0.w != f + r ||
            p_prp < lo || p_prp + ((uint64_t)p_nblk << 12) > hi || p_nblk > c.blocks_per_line) {
          raise_error(c, E_PROTO, ((uint64_t)q << 32) | s);
          p_status = 0x4;  // invalid field
        } else if (p_slba + p_nblk > c.dev_blocks) {
          p_status = 0x80;  // LBA out of range
        }
        uint64_t dl = t + c.lat_ticks;
        if (c.tok_fp) {
          const uint64_t tk = t + ((tok0 + (uint64_t)r * c.tok_fp) >> TOK_FRAC);
          if (tk > dl) dl = tk;
        }
        p_deadline = dl;
        pend = true;
      }
      freem &= ~ballot(take);
      progress = true;
    }
    tp = ptick(c, P_CTRL_FETCH, tp);
    // 2. execute ready commands: copy their blocks across PCIe
    const uint64_t tn = now();
    const uint64_t ready = ballot(pend && !p_copied && p_deadline <= tn);
    if (ready) {
      // The store image changes during a launch only through WRITE commands.  A
      // controller that copied writes releases them at system scope and then bumps the
      // image epoch; one that sees a new epoch drops its L2's copies of host memory
      // before copying (an acquire at system scope invalidates the whole L2 of its XCD,
      // which costs every wave there, so it is not done per batch).  A READ of a block
      // that was written back is submitted only after that write's completion has
      // reached the reader, so the reader sees the new epoch.
      const uint64_t ep = uni64(ld_rlx(counter(c, C_IMG_EPOCH)));
      if (ep != img_epoch) {
        fence_acq_sys();
        img_epoch = ep;
      }
      copy_cmds(c, ready, p_opc, p_nblk, p_status, p_slba, p_prp, p_q);
      if (ballot(((ready >> lane()) & 1ull) && p_opc == OPC_WRITE && !p_status)) {
        fence_rel_sys();
        if (lane() == 0) add_rel(counter(c, C_IMG_EPOCH), 1ull);
      }
      if ((ready >> lane()) & 1ull) p_copied = true;
      if (lane() == 0) count(c, C_CTRL_CMDS, __popcll(ready));
      progress = true;
    }
    // 3. post completions for executed commands, as many as each CQ has room for.  A
    //    command that does not fit stays pending; the controller never waits for CQ
    //    room (the room frees only when the completion service sees a full window,
    //    which may need the very entries this wave is holding).
    tp = ptick(c, P_CTRL_COPY, tp);
    const uint64_t done = ballot(pend && p_copied);
    if (done) {
      uint64_t todo = done;
      bool posting = false;
      uint32_t pos = 0;
      while (todo) {
        const uint32_t q = rdlane(p_q, ffs64(todo));
        const uint64_t mm = ballot(((todo >> lane()) & 1ull) && p_q == q);
        const uint32_t k = __popcll(mm);
        qp_t* qs = c.qp + q;
        uint32_t base = 0, kk = 0;
        if (lane() == 0) {
          uint32_t tail = ld_rlx(&qs->cq_tail);
          for (;;) {
            const uint32_t head = ld_rlx(&qs->cq_head);
            const uint32_t room = c.depth - (tail - head);
            kk = room < k ? room : k;
            if (kk == 0) break;
            if (!shared) {
              st_rlx(&qs->cq_tail, tail + kk);
              break;
            }
            if (cas(&qs->cq_tail, tail, tail + kk)) break;
          }
          base = tail;
        }
        base = rdlane(base, 0);
        kk = rdlane(kk, 0);
        if (((mm >> lane()) & 1ull) && mbcnt(mm) < kk) {
          pos = base + mbcnt(mm);
          cqe_t* e = c.cq + (size_t)q * c.depth + (pos & dmask);
          e->dw0 = p_line;
          e->dw1 = p_opc;
          e->dw2 = (p_cid & 0xFFFF) | (q << 16);
          posting = true;
        }
        todo &= ~mm;
      }
      const uint64_t pm = ballot(posting);
      if (pm) {
        // one release for the copied blocks (system scope when host memory was written)
        // and the entry bodies, then the phase words that make the entries visible
        if (ballot(posting && p_opc == OPC_WRITE)) fence_rel_sys(); else fence_rel();
        if (posting) {
          cqe_t* e = c.cq + (size_t)p_q * c.depth + (pos & dmask);
          const uint32_t phase = ((pos >> c.depth_shift) & 1u) ^ 1u;
          st_rlx(&e->dw3, (p_cid & 0xFFFF) | (phase << 16) | (p_status << 17));
          pend = false;
          p_copied = false;
        }
        progress = true;
      }
      if (profiling(c) && pm != done && lane() == 0) count(c, P_CTRL_NOROOM, 1);
    }
    tp = ptick(c, P_CTRL_POST, tp);
    if (!progress && profiling(c)) {
      const bool any_pend = ballot(pend) != 0;
      tp = ptick(c, any_pend ? P_CTRL_HOLD : P_CTRL_IDLE, t);
    }
    if (progress) {
      idle_since = now();
      idle_rounds = 0;
      continue;
    }
    if (!ballot(pend)) {
      if (service_should_exit(c, li)) break;
      // idle: back off (about 0.1 us doubling to about 3 us) between doorbell polls
      const uint32_t reps = idle_rounds < 5 ? (1u << idle_rounds) : 32u;
      ++idle_rounds;
      for (uint32_t r = 0; r < reps; ++r) __builtin_amdgcn_s_sleep(4);
    } else {
      // holding commands: wait on the clock alone (no memory traffic) until the earliest
      // deadline, at most about 2 us, then look at the doorbells again
      uint64_t first = ~0ull;
      if (pend && !p_copied) first = p_deadline;
      for (uint32_t o = 32; o; o >>= 1) {
        const uint64_t x = ((uint64_t)shfl32((uint32_t)(first >> 32), lane() ^ o) << 32) |
                           shfl32((uint32_t)first, lane() ^ o);
        first = x < first ? x : first;
      }
      first = uni64(first);
      const uint64_t until = now() + 200;
      const uint64_t stop = first < until ? first : until;
      while (now() < stop) __builtin_amdgcn_s_sleep(2);
    }
    if (aborted(c)) break;
    // (a held command may legitimately wait out the emulated latency first)
    if (now() - idle_since > c.timeout_ticks + c.lat_ticks) {
      if (ballot(pend)) raise_error(c, E_TIMEDOUT, 0xC1000000ull | cw);
      // idle for a whole timeout while users still run: keep waiting for them unless
      // the context was aborted (their own waits carry deadlines).
      idle_since = now();
    }
    (void)busy;
  }
}

// Completion service wavefront (Alg. 1 with a 64-entry window): CQs q = w, w + n_cq, ...
// Lane k keeps the window start and done-mask of the k-th of them in registers (they
// are also saved in the queue pair between launches).  For one CQ, lane i checks entry
// start + i against the phase expected for that lap; each new entry frees its SQ slot for
// the slot's next lap, moves its line from FETCHING to READY (or WRITEBACK to READY), and
// sets its mask bit.  When the mask is full the window advances by 64 and the CQ head
// doorbell is written.
__device__ __forceinline__ void completion(const dev_ctx& c, const launch_t& li, uint32_t w) {
  const uint32_t dmask = c.depth - 1;
  const uint32_t nmy = (c.num_qp > w) ? (c.num_qp - w + li.n_cq - 1) / li.n_cq : 0;
  if (nmy == 0) return;
  // state of my k-th CQ lives in lane k
  uint32_t off = 0;
  uint64_t mask = 0;
  if (lane() < nmy) {
    qp_t* qs = c.qp + (w + lane() * li.n_cq);
    off = ld_rlx(&qs->cq_head);
    mask = ((uint64_t)ld_rlx(&qs->cq_mask_hi) << 32) | ld_rlx(&qs->cq_mask_lo);
  }
  uint64_t idle_since = now();
  uint32_t loops = 0, idle_rounds = 0;
  for (;;) {
    if (((++loops) & 1023) == 0 && lane() == 0) count(c, C_CQ_LOOPS, 1);
    const uint64_t tl = now();
    bool any = false;
    for (uint32_t k = 0; k < nmy && k < 64; ++k) {
      const uint32_t q = w + k * li.n_cq;
      uint32_t o = rdlane(off, k);
      uint64_t mk = rdlane64(mask, k);
      const uint32_t pos = o + lane();
      bool fresh = false;
      // hint: nothing can be new while the controller's posting counter has not passed
      // the entries this window already consumed
      const uint32_t tail = uni(ld_rlx(&c.qp[q].cq_tail));
      const uint32_t seen = o + (uint32_t)__popcll(mk);
      if (tail != seen && !((mk >> lane()) & 1ull)) {
        cqe_t* e = c.cq + (size_t)q * c.depth + (pos & dmask);
        const uint32_t dw3 = ld_rlx(&e->dw3);
        const uint32_t expect = ((pos >> c.depth_shift) & 1u) ^ 1u;
        fresh = ((dw3 >> 16) & 1u) == expect;
      }
      // one acquire (the entries and the data they announce) and one release (the line
      // states that publish that data) per window visit
      const uint64_t nb = ballot(fresh);
      if (nb) {
        fence_acq();
        fence_rel();
      }
      // user buffers waiting for lines this window fills: each fresh READ closes its
      // line's pending list, and the whole wave copies the line's block into every buffer
      // on it before the line turns READY (Sec. 3.4.1)
      uint32_t plist = PEND_EMPTY, pline = 0;
      if (fresh) {
        const cqe_t* e = c.cq + (size_t)q * c.depth + (pos & dmask);
        const uint32_t line = e->dw0;
        if (e->dw1 == OPC_READ && line < c.num_lines) {
          plist = __hip_atomic_exchange(c.pend_head + line, PEND_CLOSED, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
          pline = line;
        }
      }
      if (ballot(plist < PEND_CLOSED)) {
        for (uint64_t todo = ballot(plist < PEND_CLOSED); todo; todo &= todo - 1) {
          const uint32_t l = ffs64(todo);
          const uint8_t* src = line_ptr(c, rdlane(pline, l));
          for (uint32_t en = rdlane(plist, l); en < PEND_CAP;) {
            const uint64_t dst = uni64(ld_rlx(c.pend + 2 * en));
            const uint64_t nx = uni64(ld_rlx(c.pend + 2 * en + 1));
            const uint4* s4 = reinterpret_cast<const uint4*>(src + (nx >> 32));
            uint4* d4 = reinterpret_cast<uint4*>((uintptr_t)dst);
#pragma unroll
            for (uint32_t i = 0; i < 4; ++i) d4[i * 64 + lane()] = s4[i * 64 + lane()];
            en = (uint32_t)nx;
          }
        }
        fence_rel();  // the copies before the lines turn READY
      }
      if (fresh) {
        {
          cqe_t* e = c.cq + (size_t)q * c.depth + (pos & dmask);
          const uint32_t dw3 = ld_rlx(&e->dw3);
          const uint32_t line = e->dw0;
          const uint32_t opc = e->dw1;
          const uint32_t cid = dw3 & 0xFFFF;
          const uint32_t status = dw3 >> 17;
          if (status) raise_error(c, E_IO, ((uint64_t)q << 32) | cid);
          if (line < c.num_lines) {
            if (opc == OPC_READ)
              add_rlx(c.meta + line, 1ull);  // FETCHING -> READY
            else
              add_rlx(c.meta + line, (uint64_t)0 - 2ull);  // WRITEBACK -> READY
          } else {
            raise_error(c, E_PROTO, ((uint64_t)q << 32) | cid);
          }
          uint32_t* sl = c.slot + (size_t)q * c.depth + (cid & dmask);
          const uint32_t sw = ld_rlx(sl);
          st_rlx(sl, (((sw >> 2) + c.depth) << 2) | SLOT_EMPTY);
        }
      }
      if (nb) {
        any = true;
        mk |= nb;
        if (lane() == 0) {
          add_rlx(counter(c, C_COMPLETED), (uint64_t)__popcll(nb));
          add_rlx(counter(c, C_CQ_ENTRIES), (uint64_t)__popcll(nb));
        }
        if (mk == ~0ull) {
          o += 64;
          mk = 0;
          if (lane() == 0) st_rlx(&c.qp[q].cq_head, o);
        }
        if (lane() == k) {
          off = o;
          mask = mk;
        }
      }
    }
    ptick(c, any ? P_CQ_BUSY : P_CQ_IDLE, tl);
    if (any) {
      idle_since = now();
      idle_rounds = 0;
      continue;
    }
    if (service_should_exit(c, li)) break;
    {
      // idle: back off from about 25 ns to about 0.8 us between polls
      const uint32_t reps = idle_rounds < 5 ? (1u << idle_rounds) : 32u;
      ++idle_rounds;
      for (uint32_t r = 0; r < reps; ++r) __builtin_amdgcn_s_sleep(1);
    }
    if (now() - idle_since > 4 * c.timeout_ticks) {
      // with every command completed this is an idle serving session (requests may come
      // far apart), not a lost completion
      if (uni64(ld_rlx(counter(c, C_SUBMITTED))) == uni64(ld_rlx(counter(c, C_COMPLETED)))) {
        idle_since = now();
      } else {
        raise_error(c, E_TIMEDOUT, 0xC2000000ull | w);
        break;
      }
    }
  }
  if (lane() < nmy) {
    qp_t* qs = c.qp + (w + lane() * li.n_cq);
    st_rlx(&qs->cq_mask_lo, (uint32_t)mask);
    st_rlx(&qs->cq_mask_hi, (uint32_t)(mask >> 32));
  }
}

__device__ __forceinline__ uint32_t service_role(const launch_t& li) {
  return (threadIdx.x / 64) * li.service_blocks + blockIdx.x;
}
__device__ __forceinline__ void run_service(const dev_ctx& c, const launch_t& li) {
  const uint32_t sw = service_role(li);
  if (li.prio) __builtin_amdgcn_s_setprio(3);
  if (lane() == 0 && sw < li.n_ctrl + li.n_cq) count(c, C_SVC_START, 1);
  if (sw < li.n_ctrl)
    controller(c, li, sw);
  else if (sw < li.n_ctrl + li.n_cq)
    completion(c, li, sw - li.n_ctrl);
  else
    return;
  // The launch-relative counters (user waves done, work grabbed) start every launch at
  // zero: the last service wavefront to leave clears them.  By then every user wave has
  // reported done and every other service wave has left its loop, and the next launch
  // on the stream starts after this one ends.  Nothing is tracked on the host, so a
  // launch can be captured once in a graph and replayed.
  if (lane() == 0) {
    const uint64_t n = add_acqrel(counter(c, C_SVC_EXIT), 1ull) + 1;
    if (n == (uint64_t)li.n_ctrl + li.n_cq) {
      st_rlx(counter(c, C_USER_DONE), 0ull);
      for (uint32_t p = 0; p < WORK_PARTS; ++p) st_rlx(counter(c, work_counter(p)), 0ull);
      // and the deferred count of the resident-hit pass that ran before this launch
      st_rlx(counter(c, C_DEFER), 0ull);
      st_rlx(counter(c, C_PEND), 0ull);
      st_rel(counter(c, C_SVC_EXIT), 0ull);
    }
  }
}

// Per-wavefront statistics.  The counters that user waves bump on every chunk are summed
// in the wave's own LDS slots and added to the device counters once, when the wave ends:
// thousands of waves adding to a handful of device-scope addresses would serialise there.
// The user-wave stage timers (profile flag only) are kept the same way.
enum : uint32_t {
  WS_REQUESTS = 0, WS_HITS, WS_MISSES, WS_EAGAIN, WS_AUX1, WS_WROWS,
  WS_T_ISSUE, WS_T_SUBMIT, WS_T_WAIT, WS_T_CONSUME, WS_T_DESC, WS_T_LIFE, WS_DEFLEN, WS_COUNT
};
__device__ __forceinline__ uint32_t ws_counter(uint32_t k) {
  constexpr uint32_t map[WS_COUNT] = {C_REQUESTS, C_HITS, C_MISSES, C_EAGAIN, C_AUX1, C_WROWS,
                                      P_U_ISSUE, P_U_SUBMIT, P_U_WAIT, P_U_CONSUME, P_U_DESC, P_U_LIFE,
                                      C_DEFLEN};
  return map[k];
}
struct wg_stats_t {
  uint64_t ws[WPB][WS_COUNT];  // each wave's own slots
  uint32_t waves_done;         // waves of the workgroup that have finished
};
__device__ __forceinline__ wg_stats_t& wg_stats() {
  __shared__ wg_stats_t s;
  return s;
}
__device__ __forceinline__ uint64_t* wave_stats() { return wg_stats().ws[threadIdx.x / 64]; }
// Called by every wavefront of a user workgroup (all of them, unconditionally) before
// its first chunk.
__device__ __forceinline__ void user_wave_begin() {
  if (lane() < WS_COUNT) wave_stats()[lane()] = lane() == WS_T_LIFE ? (uint64_t)0 - now() : 0;
  if (threadIdx.x == 0) wg_stats().waves_done = 0;
  __syncthreads();
}
// Lane 0 only.
__device__ __forceinline__ void wcount(uint32_t k, uint64_t v) {
  if (v) wave_stats()[k] += v;
}
// User-wave stage timer k (profile flag only): adds now() - t, returns now().
__device__ __forceinline__ uint64_t wtick(const dev_ctx& c, uint32_t k, uint64_t t) {
  if (!profiling(c)) return 0;
  const uint64_t n = now();
  if (lane() == 0) wave_stats()[k] += n - t;
  return n;
}

// Called by every user wavefront when it is done with this launch.  The last wave of the
// workgroup to finish adds the workgroup's totals to the device counters and reports
// its WPB waves done (only launches with service wavefronts count them): thousands of
// waves each adding to the same few device-scope words at the end of a launch had
// serialised there for tens of microseconds.
__device__ __forceinline__ void user_wave_done(const dev_ctx& c, const launch_t& li) {
  wg_stats_t& s = wg_stats();
  if (lane() == WS_T_LIFE) {
    uint64_t& v = wave_stats()[WS_T_LIFE];
    v = profiling(c) ? v + now() : 0;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  uint32_t n = 0;
  if (lane() == 0)
    n = __hip_atomic_fetch_add(&s.waves_done, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
  if (rdlane(n, 0) != WPB - 1) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  if (lane() < WS_COUNT) {
    uint64_t v = 0;
    for (uint32_t w = 0; w < WPB; ++w) v += s.ws[w][lane()];
    if (v) add_rlx(counter(c, ws_counter(lane())), v);
  }
  if (lane() == 0 && li.service_blocks) add_rel(counter(c, C_USER_DONE), (uint64_t)WPB);
}

// ------------------------------------------------------------------ cache (Sec. 3.4)
enum : uint32_t { A_NONE = 0, A_HIT = 1, A_JOIN = 2, A_MISS = 3, A_NEED_WB = 4, A_EAGAIN = 5 };

struct acq_t {
  uint32_t res;   // A_*
  uint32_t idx;   // cache line index (HIT/JOIN/MISS/NEED_WB)
  uint32_t gen;
};

// A set lock holds 1, or in lock-chain mode the holder's wave number + 2.
__device__ __forceinline__ bool try_lock(const dev_ctx& c, uint32_t* l) {
  uint32_t z = 0;
  return cas(l, z, lockchain(c) ? wave_gid() + 2u : 1u);
}
__device__ __forceinline__ void unlock(uint32_t* l) { st_rel(l, 0u); }

// Pins a way whose probe showed `tag` valid.  The pin is an atomic add of the pin
// count; if the word it returns no longer carries `tag` in a non-INVALID state the add is
// undone and the result is false.  Otherwise true, with res = HIT or JOIN (pinned), or
// res = EAGAIN when the line already holds RC_LIMIT pins (the add is undone).
__device__ __forceinline__ bool pin_way(const dev_ctx& c, uint32_t idx, uint32_t tag, uint32_t cnt,
                                        uint32_t& res, uint32_t& gen) {
  const uint64_t old = add_rlx(c.meta + idx, RC_ONE * cnt);
  if (m_tag(old) == tag && m_state(old) != ST_INVALID) {
    if (m_rc(old) + cnt > RC_LIMIT) {  // the line holds as many pins as it may: EAGAIN
      add_rlx(c.meta + idx, (uint64_t)0 - RC_ONE * cnt);
      res = A_EAGAIN;
      return true;
    }
    res = (m_state(old) == ST_FETCHING) ? A_JOIN : A_HIT;
    gen = m_gen(old);
    if (!(old & M_REF)) or_rlx(c.meta + idx, M_REF);
    return true;
  }
  add_rlx(c.meta + idx, (uint64_t)0 - RC_ONE * cnt);
  return false;
}

// One acquisition attempt for `line_id` by this lane, pinning `cnt` references.
//  * HIT / JOIN: the tag is present (READY, DIRTY, WRITEBACK / FETCHING): pinned.
//  * MISS: a victim was claimed as FETCHING(line_id) with the pins; the caller must
//    submit the READ.
//  * NEED_WB: the clock chose a DIRTY victim; it is now WRITEBACK with one pin of ours;
//    the caller submits its WRITE, waits for it, and calls again with `retake` = the line.
//  * EAGAIN: every way is pinned or in flight (cache deadlock avoidance, Sec. 2.3.2).
// Misses take the set lock so that a tag is never inserted twice; hits never lock.
// Probes a set for `tag`: every way's metadata word is loaded before any is compared
// (16 device-coherent loads in flight per lane), so a probe costs one round trip for up
// to 16 ways.  Returns the way or -1, and the word seen.
__device__ __forceinline__ int probe_set(const dev_ctx& c, uint32_t base, uint32_t tag, uint64_t& seen) {
  for (uint32_t g = 0; g < c.assoc; g += 16) {
    uint64_t w[16];
#pragma unroll
    for (uint32_t i = 0; i < 16; ++i) w[i] = (g + i < c.assoc) ? ld_rlx(c.meta + base + g + i) : 0ull;
    int f = -1;
#pragma unroll
    for (uint32_t i = 0; i < 16; ++i)
      if (f < 0 && g + i < c.assoc && m_tag(w[i]) == tag && m_state(w[i]) != ST_INVALID) {
        f = (int)(g + i);
        seen = w[i];
      }
    if (f >= 0) return f;
  }
  return -1;
}

// LDS-staged probe of a whole wave's sets (level-2 coalescing, Sec. 3.3.2 / Sec. 3.4).
// A lane-per-lookup probe reads its set with one load per way, so one wave instruction
// touches 64 different metadata lines; here the wave instead copies the sets of its
// lookups into LDS with 16-byte global-to-LDS loads, each instruction moving 64 / (A/2)
// whole sets of A 8-byte words (A = assoc) as contiguous bytes: one request per
// metadata line instead of one per word.  Then every lane compares its own set's words
// in LDS.  The loads bypass registers (LDS DMA) and are device-coherent.  The copies land
// set-major (set t of the pass at 8A * t), and a lane reads its set's 16-byte pairs in an
// order rotated by its slot, so that the eight lanes the LDS serves together read eight
// different 16-byte columns of the 128-byte bank row.
constexpr uint32_t PROBE_LDS = 8192;  // bytes of LDS per wavefront
struct alignas(16) probe_lds_t {
  uint8_t b[WPB][PROBE_LDS];
};
__device__ __forceinline__ uint8_t* probe_area() {
  __shared__ probe_lds_t s;
  return s.b[threadIdx.x / 64];
}
// Sets of one load pass: 8 KiB of LDS per wave holds 1024 / A sets.
__host__ __device__ constexpr bool probe_staged_ok(uint32_t assoc) {
  return assoc >= 2 && assoc <= 64 && (assoc & (assoc - 1)) == 0;
}
typedef __attribute__((address_space(3))) void lds_void;
typedef unsigned int lds_u32x4_t __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) lds_u32x4_t lds_u32x4;

// Lanes with `want` probe the set starting at line index `base` for `tag`; returns the
// way (or -1) and the word seen.  Every lane of the wave must call it.
__device__ __forceinline__ int probe_staged(const dev_ctx& c, bool want, uint32_t base, uint32_t tag,
                                            uint64_t& seen, uint8_t* lds) {
  const uint32_t A = c.assoc;
  const uint32_t P = A / 2;                            // 16-byte pairs per set
  const uint32_t pl = (uint32_t)__builtin_ctz(P);      // log2 P
  const uint32_t per = A <= 16 ? 64u : 1024u / A;      // sets per pass
  const uint32_t spi = 64u >> pl;                      // sets per load instruction
  const uint32_t rl = P >= 8 ? 0u : 3u - pl;           // log2 of the slots per rotation step
  const uint32_t me = lane();
  const uint64_t wm = ballot(want);
  int way = -1;
  for (uint32_t s0 = 0; s0 < 64; s0 += per) {
    if (!((wm >> s0) & (per == 64 ? ~0ull : ((1ull << per) - 1ull)))) continue;
    const uint32_t ninstr = per / spi;
    for (uint32_t i = 0; i < ninstr; ++i) {
      const uint32_t t = i * spi + (me >> pl);  // slot within the pass
      const uint32_t sb = shfl32(base, s0 + t);
      if ((wm >> (s0 + t)) & 1ull) {
        const uint64_t* src = c.meta + sb + 2 * (me & (P - 1));
        __builtin_amdgcn_global_load_lds((const void*)src, (lds_void*)(lds + i * 1024u), 16, 0,
                                         16 /* sc1: device-coherent */);
      }
    }
    // the LDS copies have landed once this wave's vector memory counter drains; the
    // empty asm keeps the compiler from moving the LDS reads above the wait
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    asm volatile("" ::: "memory");
    const uint32_t t = me - s0;
    if (want && me >= s0 && me < s0 + per) {
      const uint32_t rot = t >> rl;
      const uint8_t* row = lds + t * 8u * A;
      for (uint32_t j0 = 0; j0 < P && way < 0; j0 += 4) {
        lds_u32x4_t v[4];
#pragma unroll
        for (uint32_t u = 0; u < 4; ++u)
          if (j0 + u < P) v[u] = *(const lds_u32x4*)(row + 16u * ((j0 + u + rot) & (P - 1)));
#pragma unroll
        for (uint32_t u = 0; u < 4; ++u) {
          if (j0 + u >= P || way >= 0) continue;
          const uint32_t p = (j0 + u + rot) & (P - 1);
          const uint64_t w0 = ((uint64_t)v[u].y << 32) | v[u].x;
          const uint64_t w1 = ((uint64_t)v[u].w << 32) | v[u].z;
          if (m_tag(w0) == tag && m_state(w0) != ST_INVALID) {
            way = (int)(2 * p);
            seen = w0;
          } else if (m_tag(w1) == tag && m_state(w1) != ST_INVALID) {
            way = (int)(2 * p + 1);
            seen = w1;
          }
        }
      }
    }
  }
  // the next staged probe of this wave overwrites the area: its reads above are done
  // (their values were used), and no other wave touches it
  return way;
}

// `cnt` == 0 asks for an unpinned hit: a resident or in-flight line is reported with its
// generation and not pinned (the caller validates after reading); a miss still pins its
// claim with one reference, unless !pin_miss (a prefetch: the claim is FETCHING with no
// reference, which no eviction takes, and once filled it is an ordinary unpinned line).
__device__ __forceinline__ acq_t acquire_try(const dev_ctx& c, uint32_t line_id, uint32_t cnt, int retake,
                                             bool pin_miss = true) {
  acq_t r{A_NONE, 0, 0};
  const uint32_t set = set_of(c, line_id);
  const uint32_t base = set * c.assoc;
  const bool pin_hits = cnt != 0;
  if (cnt == 0 && pin_miss) cnt = 1;
  if (retake < 0) {
    // lock-free probe
    uint64_t m = 0;
    const int w = probe_set(c, base, line_id, m);
    if (w >= 0) {
      if (!pin_hits) {
        r.res = (m_state(m) == ST_FETCHING) ? A_JOIN : A_HIT;
        r.gen = m_gen(m);
        r.idx = base + (uint32_t)w;
        if (!(m & M_REF)) or_rlx(c.meta + r.idx, M_REF);
        return r;
      }
      if (pin_way(c, base + (uint32_t)w, line_id, cnt, r.res, r.gen)) {
        r.idx = base + (uint32_t)w;
        return r;
      }
    }
  }
  if (!try_lock(c, c.set_lock + set)) return r;  // A_NONE: retry later
  // re-probe under the lock: tags only change while the lock is held
  for (uint32_t w = 0; w < c.assoc; ++w) {
    const uint64_t m = ld_rlx(c.meta + base + w);
    if (m_tag(m) == line_id && m_state(m) != ST_INVALID) {
      if (!pin_hits) {
        r.res = (m_state(m) == ST_FETCHING) ? A_JOIN : A_HIT;
        r.gen = m_gen(m);
        r.idx = base + w;
        if (!(m & M_REF)) or_rlx(c.meta + r.idx, M_REF);
        if (retake >= 0) add_rel(c.meta + retake, (uint64_t)0 - RC_ONE);
        unlock(c.set_lock + set);
        return r;
      }
      if (pin_way(c, base + w, line_id, cnt, r.res, r.gen)) {
        r.idx = base + w;
        if (retake >= 0) add_rel(c.meta + retake, (uint64_t)0 - RC_ONE);  // drop our WB pin
        unlock(c.set_lock + set);
        return r;
      }
    }
  }
  if (retake >= 0) {
    // our written-back line: READY(old tag) holding exactly our one pin -> FETCHING(new)
    uint64_t m = ld_rlx(c.meta + retake);
    if (m_state(m) == ST_READY && m_rc(m) == 1) {
      const uint64_t nw = ((uint64_t)line_id << TAG_SHIFT) |
                          ((uint64_t)((m_gen(m) + 1) & 0xFF) << GEN_SHIFT) | (RC_ONE * cnt) |
                          M_REF | ST_FETCHING;
      if (cas(c.meta + retake, m, nw)) {
        st_rlx(c.pend_head + retake, PEND_EMPTY);
        r.res = A_MISS;
        r.idx = retake;
        r.gen = (m_gen(m) + 1) & 0xFF;
        unlock(c.set_lock + set);
        return r;
      }
    }
    add_rel(c.meta + retake, (uint64_t)0 - RC_ONE);
  }
  // clock sweep from the hand (second chance); pinned / in-flight ways are skipped
  const uint32_t h0 = ld_rlx(c.hand + set);
  uint32_t h = h0;
  for (uint32_t step = 0; step < 2 * c.assoc + 1; ++step) {
    const uint32_t idx = base + h;
    uint64_t m = ld_rlx(c.meta + idx);
    const uint32_t st = m_state(m);
    const bool unpinned = m_rc(m) == 0;
    bool victim = false, dirty = false;
    if (st == ST_INVALID) {
      victim = true;
    } else if ((st == ST_READY || st == ST_DIRTY) && unpinned) {
      if (m & M_REF) {
        and_rlx(c.meta + idx, ~M_REF);
      } else {
        victim = true;
        dirty = st == ST_DIRTY;
      }
    }
    if (victim) {
      uint64_t nw;
      if (dirty) {
        nw = (m & ~(M_STATE | M_REF | RC_MASK)) | RC_ONE | ST_WRITEBACK;
      } else {
        nw = ((uint64_t)line_id << TAG_SHIFT) | ((uint64_t)((m_gen(m) + 1) & 0xFF) << GEN_SHIFT) |
             (RC_ONE * cnt) | M_REF | ST_FETCHING;
      }
      if (cas(c.meta + idx, m, nw)) {
        if (!dirty) st_rlx(c.pend_head + idx, PEND_EMPTY);  // a new tenant: no waiting buffers yet
        st_rlx(c.hand + set, (h + 1) % c.assoc);
        r.res = dirty ? A_NEED_WB : A_MISS;
        r.idx = idx;
        r.gen = dirty ? m_gen(m) : ((m_gen(m) + 1) & 0xFF);
        unlock(c.set_lock + set);
        return r;
      }
      continue;  // lost a race on this way: look at it again
    }
    h = (h + 1) % c.assoc;
  }
  st_rlx(c.hand + set, h);
  unlock(c.set_lock + set);
  r.res = A_EAGAIN;
  return r;
}

// ------------------------------------------------------------------ wave request chunks
// A chunk is up to 64 lookups, one per lane.  issue() coalesces duplicate lines within the
// wave (level-1 coalescing, Sec. 3.3.2: one leader lane per distinct line), acquires the
// leaders' lines (level-2 coalescing in the cache), submits the wave's READs with one
// reservation, and broadcasts each leader's line to its followers.  Optimistic readers
// probe first and coalesce only the lanes whose line is neither resident nor in flight:
// a hit needs no leader, since it issues nothing.
// Pinning modes of a chunk.
enum : uint32_t {
  PIN_LINE = 0,  // one pin per distinct line (writers, serialized traces)
  PIN_EACH = 1,  // one pin per lane (host tickets)
  PIN_NONE = 2,  // optimistic readers: hits are not pinned, a wave's own misses are
  PIN_PREFETCH = 3  // prefetch (Listing 1's prefetch()): nothing is pinned, a full set
                    // drops the lane's request, and the caller neither waits nor releases
};

struct chunk_t {
  uint32_t line_id;  // requested line (valid when act)
  uint32_t off;      // byte offset inside the line
  uint32_t idx;      // cache line index (valid when st == A_HIT/JOIN/MISS)
  uint32_t st;       // A_* result for this lane (followers copy their leader)
  uint32_t leader;   // leader lane of this lane's line
  uint32_t cnt;      // leader: lanes sharing its line
  uint32_t gen;      // generation of the line when acquired
  bool act;          // this lane carries a lookup
  bool pinned;       // this lane's line holds a pin taken by this chunk
};

__device__ __forceinline__ bool st_ok(uint32_t st) {
  return st == A_HIT || st == A_JOIN || st == A_MISS;
}

// Leader election among the lanes with `part` (the others lead themselves).
__device__ __forceinline__ void dedup(chunk_t& ch, bool part) {
  uint64_t todo = ballot(part);
  ch.leader = lane();
  ch.cnt = 0;
  while (todo) {
    const uint32_t l = ffs64(todo);
    const uint32_t v = rdlane(ch.line_id, l);
    const uint64_t same = ballot(part && ch.line_id == v);
    if ((same >> lane()) & 1ull) ch.leader = l;
    if (lane() == l) ch.cnt = __popcll(same);
    todo &= ~same;
  }
}

// Acquire + submit for the leaders of `ch`.  On return every active lane has st in
// {A_HIT, A_JOIN, A_MISS, A_EAGAIN} (or the context aborted).  Counts stats.
// `probe_first` (optimistic readers only) suits lanes that mostly want distinct lines
// (embedding rows); readers whose lanes share lines (consecutive CSR entries) coalesce
// first and probe once per distinct line.
__device__ __forceinline__ bool chunk_issue(const dev_ctx& c, chunk_t& ch, uint32_t q, bool count_stats,
                            uint32_t pin_mode = PIN_LINE, bool probe_first = true, bool fetch = true) {
  const uint64_t t_issue = now();
  uint32_t st = A_NONE, idx = 0, gen = 0;
  bool part = ch.act;  // lanes that go through dedup and the acquire loop
  const bool pf = pin_mode == PIN_PREFETCH;
  if ((pin_mode == PIN_NONE || pf) && probe_first) {
    // optimistic readers: every lane first probes its own set; a resident or in-flight
    // line is taken unpinned on the spot, and only the lanes left over elect leaders
    const uint32_t base = ch.act ? set_of(c, ch.line_id) * c.assoc : 0u;
    uint64_t m = 0;
    int w = -1;
    if (probe_staged_ok(c.assoc))
      w = probe_staged(c, ch.act, base, ch.line_id, m, probe_area());
    else if (ch.act)
      w = probe_set(c, base, ch.line_id, m);
    if (ch.act && w >= 0) {
      st = (m_state(m) == ST_FETCHING) ? A_JOIN : A_HIT;
      idx = base + (uint32_t)w;
      gen = m_gen(m);
      if (!(m & M_REF)) or_rlx(c.meta + idx, M_REF);
      part = false;
    }
  }
  dedup(ch, part);
  const bool lead = part && ch.leader == lane();
  const uint32_t npin = pin_mode == PIN_EACH ? ch.cnt : (pin_mode == PIN_LINE ? 1u : 0u);
  int retake = -1;
  bool pending = lead;
  spin_t sp;
  while (ballot(pending)) {
    bool wb = false, rd = false;
    if (pending) {
      const acq_t a = acquire_try(c, ch.line_id, npin, retake, !pf);
      if (a.res != A_NONE) {
        st = a.res;
        idx = a.idx;
        gen = a.gen;
        if (a.res == A_NEED_WB) {
          wb = true;
          retake = (int)a.idx;
        } else {
          pending = false;
          rd = a.res == A_MISS && fetch;
        }
      }
    }
    // one wave-wide submission per round and device; READs and WRITEs may share the
    // queue pair
    uint32_t lid = ch.line_id;
    if (wb) lid = m_tag(ld_rlx(c.meta + idx));
    const uint64_t ts = now();
    if (!submit_line(c, q, rd, OPC_READ, idx, lid)) return false;
    if (!submit_line(c, q, wb, OPC_WRITE, idx, lid)) return false;
    wtick(c, WS_T_SUBMIT, ts);
    if (ballot(wb)) {
      const uint64_t nwb = __popcll(ballot(wb));
      if (lane() == 0) count(c, C_WB_EVICT, nwb);
      // wait for our write-backs to finish before retaking the line
      spin_t sw;
      bool waiting = wb;
      while (ballot(waiting)) {
        if (waiting && m_state(ld_rlx(c.meta + idx)) != ST_WRITEBACK) waiting = false;
        if (ballot(waiting) && !sw.step(c, wi(W_WB, idx))) return false;
      }
      fence_acq();
    }
    if (ballot(pending && st == A_NONE)) {
      if (!sp.step(c, wi(W_SETLOCK, rdlane(ch.line_id, ffs64(ballot(pending && st == A_NONE)))))) return false;
    }
  }
  const bool pin = lead && !pf && (npin ? st_ok(st) : st == A_MISS);
  // broadcast to followers
  const uint32_t lst = shfl32(st, ch.leader);
  const uint32_t lidx = shfl32(idx, ch.leader);
  const uint32_t lgen = shfl32(gen, ch.leader);
  const uint32_t lpin = shfl32(pin ? 1u : 0u, ch.leader);
  if (ch.act) {
    ch.st = lst;
    ch.idx = lidx;
    ch.gen = lgen;
    ch.pinned = lpin != 0;
  } else {
    ch.st = A_NONE;
    ch.pinned = false;
  }
  wtick(c, WS_T_ISSUE, t_issue);
  if (count_stats) {
    const uint64_t nreq = __popcll(ballot(ch.act && ch.st != A_EAGAIN));
    const uint64_t nmiss = __popcll(ballot(ch.act && ch.st == A_MISS));
    const uint64_t nea = __popcll(ballot(lead && st == A_EAGAIN));
    if (lane() == 0) {
      wcount(WS_REQUESTS, nreq);
      wcount(WS_MISSES, nmiss);
      wcount(WS_HITS, nreq - nmiss);
      wcount(WS_EAGAIN, nea);
    }
  }
  return true;
}

// Waits until the chunk's in-flight lines have been filled: a lane waits while its line
// still carries its tag and generation in the FETCHING state.  With `acquire`, one
// acquire fence follows (plain loads of the line data are then safe); without it the
// caller reads the data with device-coherent loads.
__device__ __forceinline__ bool chunk_wait(const dev_ctx& c, const chunk_t& ch, bool acquire = true) {
  const uint64_t t_wait = now();
  // one poller per distinct line (the dedup leader); followers share its line
  bool waiting = ch.act && ch.leader == lane() && (ch.st == A_JOIN || ch.st == A_MISS);
  spin_t sp;
  while (true) {
    if (waiting) {
      const uint64_t m = ld_rlx(c.meta + ch.idx);
      if (m_state(m) != ST_FETCHING || m_tag(m) != ch.line_id || m_gen(m) != ch.gen) waiting = false;
    }
    if (!ballot(waiting)) break;
    if (!sp.step(c, wi(W_FILL, rdlane(ch.idx, ffs64(ballot(waiting)))))) return false;
  }
  if (acquire) fence_acq();
  wtick(c, WS_T_WAIT, t_wait);
  return true;
}

// True when the line of this lane still holds the data the chunk saw: same tag and
// generation, in a state with valid data.  Loaded device-coherently after the caller's
// data loads have completed.
__device__ __forceinline__ bool line_still_valid(const dev_ctx& c, uint32_t idx, uint32_t tag,
                                                 uint32_t gen) {
  const uint64_t m = ld_rlx(c.meta + idx);
  const uint32_t st = m_state(m);
  return m_tag(m) == tag && m_gen(m) == gen &&
         (st == ST_READY || st == ST_DIRTY || st == ST_WRITEBACK);
}

// Lock-chain report (flag FLAG_LOCKCHAIN; the lock-chain debugger of Sec. 3.5, for this
// library's waits): starting at wave w0 waiting for `what`, follows a set lock to the
// wave that holds it and on to what that wave waits for, until a wait on something no
// wave holds (a fill, a write-back, an SQ slot, a free way), a wave that is not waiting,
// or a wave already in the chain (a cycle).  Each hop records (wave, what, the object's
// word: the lock word, the line's metadata or the slot word) in c.chain; the first
// report of a launch wins.  One lane calls it.
__device__ void lc_walk(const dev_ctx& c, uint32_t w0, uint64_t what) {
  uint64_t z = 0;
  if (!cas(c.chain, z, 1ull)) return;
  uint32_t w = w0, n = 0;
  uint64_t seen[LC_MAX];
  bool cycle = false;
  while (n < LC_MAX) {
    const uint32_t kind = (uint32_t)(what >> 56);
    const uint64_t id = what & ((1ull << 56) - 1);
    uint64_t word = 0;
    uint32_t next = ~0u;
    if (kind == W_SETLOCK) {
      word = ld_rlx(c.set_lock + set_of(c, (uint32_t)id));
      if (word >= 2) next = (uint32_t)word - 2;
    } else if ((kind == W_WB || kind == W_FILL || kind == W_TICKET || kind == W_CLAIM) && id < c.num_lines) {
      word = ld_rlx(c.meta + id);
    } else if (kind == W_SQ_SLOT && (id >> 32) < c.num_qp) {
      word = ld_rlx(c.slot + (size_t)(id >> 32) * c.depth + ((uint32_t)id & (c.depth - 1)));
    }
    st_rlx(c.chain + 1 + 3 * n, (uint64_t)w);
    st_rlx(c.chain + 2 + 3 * n, what);
    st_rlx(c.chain + 3 + 3 * n, word);
    seen[n] = w;
    ++n;
    if (next == ~0u || next >= WAIT_SLOTS) break;
    for (uint32_t k = 0; k < n; ++k)
      if (seen[k] == next) cycle = true;
    if (cycle) {
      st_rlx(c.chain + 1 + 3 * n, (uint64_t)next);  // the wave the cycle returns to
      break;
    }
    w = next;
    what = ld_rlx(c.waits + 2 * w);
    if (what && now() - ld_rlx(c.waits + 2 * w + 1) > LC_FRESH) what = 0;
    if (!what) {  // the holder is not waiting: record it and stop
      st_rlx(c.chain + 1 + 3 * n, (uint64_t)w);
      st_rlx(c.chain + 2 + 3 * n, 0ull);
      st_rlx(c.chain + 3 + 3 * n, 0ull);
      ++n;
      break;
    }
  }
  fence_rel();
  st_rlx(c.chain, (1ull << 63) | ((uint64_t)n << 1) | (cycle ? 1ull : 0ull));
}

// Drops the pins the chunk holds (leaders only).
__device__ __forceinline__ void chunk_release(const dev_ctx& c, chunk_t& ch, bool wrote) {
  const bool lead = ch.act && ch.leader == lane() && ch.pinned;
  if (wrote) {
    if (lead) add_rel(c.meta + ch.idx, (uint64_t)0 - RC_ONE);
  } else {
    loads_done();
    if (lead) add_rlx(c.meta + ch.idx, (uint64_t)0 - RC_ONE);
  }
  ch.act = false;
}

}  // namespace ag
