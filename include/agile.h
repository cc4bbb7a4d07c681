/*
 * agile.h - C ABI of an MI355X (gfx950) library for GPU-initiated asynchronous block
 * reads through NVMe-style submission/completion queue pairs into a set-associative
 * HBM software cache (AGILE, arXiv 2504.19365).
 *
 * Model.  A store is a byte image of 4 KiB blocks in host-pinned memory.  It sits
 * behind an emulated NVMe controller that runs as GPU service wavefronts: they fetch
 * commands from submission queues (SQ) after their doorbell moves, hold each command
 * for a configurable latency and an IOPS cap, copy the block across PCIe into its HBM
 * cache line (or back, for write-back) and post a phase-tagged completion entry (CQE)
 * (Sec. 2.1).  Completion-service wavefronts consume CQEs and free SQ slots, so user
 * waves never process completions (Sec. 3.2, Alg. 1).  User waves coalesce duplicate
 * requests within a wavefront, probe the cache, and submit misses with one atomic per
 * wavefront, serialising the doorbell as in Sec. 3.3.1 / Alg. 2.  Cache lines follow
 * the INVALID / BUSY / READY / MODIFIED states of Sec. 3.4 with clock replacement.
 *
 * Every kernel this library launches carries its own service wavefronts as its first
 * workgroups, so the queues make progress during every launch without relying on two
 * kernels running side by side.  Calls on one context must not overlap in time (the
 * library is not thread-safe per context; use one stream per context).
 *
 * Conventions.  Every function returns agile_status (0 = AGILE_OK, < 0 error).
 * "Device pointer" means memory the GPU can dereference (hipMalloc or torch CUDA
 * tensors); "stream" is a hipStream_t passed as void* (NULL = default stream).
 * Calls that launch work are stream-ordered and return at once; errors raised on the
 * device latch into a sticky error word that the next blocking call (agile_wait,
 * agile_flush, agile_sync, agile_close_store) returns.  After a sticky error the
 * context accepts only agile_get_stats, agile_last_error and agile_shutdown.
 */
#ifndef AGILE_H
#define AGILE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum agile_status {
  AGILE_OK = 0,
  AGILE_EINVAL = -1,    /* bad argument or configuration; nothing was launched */
  AGILE_ENOMEM = -2,    /* device or pinned host allocation failed */
  AGILE_EHIP = -3,      /* a HIP runtime call failed */
  AGILE_ETIMEDOUT = -4, /* a device wait exceeded timeout_ns (watchdog) */
  AGILE_EAGAIN = -5,    /* no room yet (a ticket found no evictable way in its set; a session
                           is full, or a request has not completed); retry later */
  AGILE_EIO = -6,       /* a command completed with an error status */
  AGILE_EPROTO = -7,    /* queue-protocol violation detected on the device */
  AGILE_ESTATE = -8     /* call not allowed in the current state */
} agile_status;

typedef struct agile_ctx_s* agile_ctx;
typedef struct agile_store_s* agile_store;

/* A ticket names one pinned cache line: bits 0-31 line index, 32-39 generation,
 * 40-47 status (0 = ok, 1 = EAGAIN, 2 = not issued), 48-63 byte offset of the block
 * within the line divided by 4096.  Tickets live in device memory. */
typedef uint64_t agile_ticket;

/* agile_config.flags */
#define AGILE_F_SERIALIZED 0x1u /* workloads run one request at a time on one lane */
#define AGILE_F_NO_PRIO 0x2u    /* do not raise the service wavefronts' issue priority */
#define AGILE_F_PROFILE 0x4u    /* accumulate per-stage timers (see agile_debug_counters) */
#define AGILE_F_LOCKCHAIN 0x8u  /* lock-chain debugging (Sec. 3.5's lock-chain debugger for
                                   this library's waits): every spinning wavefront records
                                   what it waits for and set locks record their holder; the
                                   first wait to time out follows the chain (a set lock to
                                   its holder, to what that holder waits for, ...) and the
                                   error text of the next blocking call lists it, ending at
                                   a wait on no wave (a fill, a write-back, an SQ slot, a free
                                   way), a running wave, or a cycle */

typedef struct agile_config {
  uint32_t struct_size;  /* sizeof(agile_config) */
  int32_t device;        /* HIP device ordinal */
  uint64_t cache_bytes;  /* HBM software-cache capacity; multiple of line_bytes */
  uint32_t line_bytes;   /* 4096 << k; a line holds line_bytes/4096 consecutive blocks */
  uint32_t assoc;        /* ways per set; (cache_bytes / line_bytes) % assoc == 0 */
  uint32_t num_qp;       /* queue pairs, 1..1024 */
  uint32_t qp_depth;     /* entries per SQ and per CQ: power of two in [64, 65536] */
  uint32_t ctrl_waves;   /* emulated-controller wavefronts (0 = max(num_qp, 64)) */
  uint32_t cq_waves;     /* completion-service wavefronts (0 = min(num_qp, 64)) */
  uint32_t max_user_waves; /* cap on user wavefronts per launch (0 = fill the GPU) */
  uint64_t latency_ns;   /* emulated per-command latency, fetch to completion */
  uint64_t iops_cap;     /* emulated commands per second over the store (0 = none) */
  uint64_t timeout_ns;   /* device watchdog for every wait (0 = 10 s) */
  uint32_t flags;        /* AGILE_F_* */
  uint32_t reserved;
} agile_config;

/* Fills a configuration with defaults (1 MiB cache of 4 KiB lines, 8-way, 1 QP of 64
 * entries, no latency, no cap).  Always succeeds. */
void agile_config_default(agile_config* cfg);

/* Roughly AGILE_HOST + initializeAgile + startAgile of Listing 1 (Sec. 3.5): selects the
 * device and allocates the cache lines, per-line metadata, clock hands, SQ/CQ rings,
 * slot states, counters and the error word in HBM.  Validates cfg first and returns
 * AGILE_EINVAL without touching the GPU when it is inconsistent.  Owns everything it
 * allocates; release with agile_shutdown. */
agile_status agile_init(const agile_config* cfg, agile_ctx* out);

/* Roughly stopAgile: waits for the device to go idle and frees the context.
 * Open stores are closed without a flush. */
agile_status agile_shutdown(agile_ctx ctx);

/* Pinned, device-mapped host memory for store images (hipHostMalloc, non-coherent so
 * that the GPU reads it in whole cache lines).  The caller owns it and frees it with
 * agile_host_free after closing any store on it.  Host writes to it must happen while
 * no kernel of the context runs. */
agile_status agile_host_alloc(uint64_t bytes, void** out);
agile_status agile_host_free(void* p);

/* Roughly addNvmeDev + initNvme (Sec. 3.5): opens a store over `host_image`, which must
 * be pinned host memory the device can map (agile_host_alloc or torch pin_memory) and
 * stay valid until agile_close_store.  bytes must be a multiple of block_bytes, which
 * must be 4096.  One store per context at a time (AGILE_ESTATE otherwise). */
agile_status agile_open_store(agile_ctx ctx, void* host_image, uint64_t bytes,
                              uint32_t block_bytes, uint32_t flags, agile_store* out);

/* Several emulated devices behind one store (Sec. 4.3's multi-SSD setup: request i goes
 * to device i mod n).  The store is striped one cache line at a time: line l of the
 * store (bytes [l*line_bytes, (l+1)*line_bytes)) is line l / n of device l mod n, whose
 * image is host_images[l mod n] (each pinned as for agile_open_store, bytes_each bytes,
 * a multiple of the context's line_bytes when n > 1).  The store holds n * bytes_each
 * bytes.  Each device has its own emulated latency and its own IOPS cap (the config's
 * latency_ns and iops_cap apply per device), and owns the queue pairs q with
 * q mod n == its number (num_qp must be a multiple of n).  1 <= n <= AGILE_MAX_DEVICES;
 * agile_open_store is the case n = 1.  Same ownership and errors as agile_open_store. */
#define AGILE_MAX_DEVICES 8
agile_status agile_open_store_striped(agile_ctx ctx, void* const* host_images, uint32_t n,
                                      uint64_t bytes_each, uint32_t block_bytes, uint32_t flags,
                                      agile_store* out);

/* Roughly closeNvme: blocks until idle, invalidates the cache (dirty lines are NOT
 * written back; call agile_flush first) and detaches the store.  Returns the sticky
 * error, if any. */
agile_status agile_close_store(agile_ctx ctx, agile_store store);

/* prefetch() of Sec. 3.1 / Listing 1: for each of the n block ids in d_blocks (device
 * uint64), coalesces duplicates within a wavefront, looks up the cache and, on a miss,
 * claims a line and submits a READ.  Writes one ticket per block to d_tickets (device).
 * Each successful ticket pins its line until agile_release; a ticket whose set has no
 * evictable way, or whose line already holds 262,144 pins, carries status EAGAIN and pins
 * nothing.  Stream-ordered and returns at
 * once to the host.  Unlike the paper's prefetch(), whose reads proceed beside the
 * calling kernel, the reads of this call complete within its own kernel launch (the
 * launch carries the service wavefronts that drain every command, see the note at the
 * top): a user kernel queued after it on the same stream starts once the blocks are in
 * HBM, so host-level tickets overlap I/O with host work and with other streams, not with
 * a later kernel on this stream.  Overlap of I/O with compute inside one kernel is what
 * the library's workload entry points do (AGILE_MODE_ASYNC). */
agile_status agile_async_read(agile_ctx ctx, agile_store store, const uint64_t* d_blocks,
                              uint32_t n, agile_ticket* d_tickets, void* stream);

/* The barrier wait of Sec. 3.2 (Fig. 3) / AgileBufPtr::wait of Listing 1: waits until the
 * line of every ticket is READY and writes the device address of each ticket's 4 KiB
 * block to d_ptrs[i] (device; NULL for EAGAIN tickets).  Blocks the host until the
 * stream is idle.  Returns the sticky error if any, else AGILE_EAGAIN if any ticket
 * carried EAGAIN, else AGILE_OK. */
agile_status agile_wait(agile_ctx ctx, const agile_ticket* d_tickets, uint32_t n, void** d_ptrs,
                        void* stream);

/* Ends the use of n tickets' lines: drops the pin each ticket holds, so the line may be
 * evicted again.  A line in use must not be evicted before its accesses are done, and
 * pins that are never dropped are what deadlocks a software cache (Sec. 2.3.2); a line
 * is only evicted in the READY/MODIFIED states once nobody holds it (Sec. 3.4 case d).
 * EAGAIN tickets (which pin nothing) are skipped.  d_tickets is device memory written by
 * agile_async_read; releasing a ticket twice is an error the library does not detect.
 * Stream-ordered. */
agile_status agile_release(agile_ctx ctx, const agile_ticket* d_tickets, uint32_t n,
                           void* stream);

/* Writes every MODIFIED (dirty) line back to the store exactly once and leaves it clean
 * (Sec. 3.4 case d).  Requires that no line is pinned.  Blocks until done and returns
 * the sticky error, if any. */
agile_status agile_flush(agile_ctx ctx, agile_store store, void* stream);

/* The write of Sec. 3.5's API (asyncWrite: through the cache; the caller's buffer may
 * be reused once the call is done), for whole lines: line d_lines[i] (device uint64,
 * a line id < the store's lines) takes line_bytes bytes from d_src + i * line_bytes
 * (device memory).  Each line is found in the cache or allocated without a read (a
 * dirty victim is written back first), filled, and written to its device by one WRITE
 * command before the call returns (write-through); the cached copy stays, clean.  Of
 * entries that name the same line, the one at the highest i within a wavefront's 64 is
 * written; across wavefronts the order is unspecified.  The store must hold whole
 * lines.  Blocks until done; returns the sticky error, if any. */
agile_status agile_write(agile_ctx ctx, agile_store store, const uint64_t* d_lines, uint32_t n,
                         const void* d_src, void* stream);

/* Reads into user buffers with the Share Table (Sec. 3.4.1; Listing 1's asyncRead into an
 * AgileBuf).  Request i delivers store block d_blocks[i] (device uint64, < the store's
 * blocks) into the caller's buffer d_bufs[i] (device memory, 4096 bytes, 16-byte
 * aligned).  A block resident in the cache is copied at once; a block whose line is being
 * filled puts the buffer on the line's pending list and the completion service copies
 * the block into it before the line turns READY, so the requesting wavefront goes on to
 * its next requests instead of waiting (the buffer, not a cache line, holds the data
 * afterwards: no pin is kept).  With AGILE_ISSUE_SHARE the Share Table is consulted
 * first: the first live holder of a block owns it (status AGILE_BUF_OWNER, its buffer
 * receives the block) and later requests for the same block share the owner's buffer
 * (AGILE_BUF_SHARED: d_ptrs[i] points at it, no copy is made) until every holder has
 * released it (agile_buffers_release); a block that finds no free table slot along its
 * probe is copied privately (AGILE_BUF_PRIVATE, as without the flag).  d_ptrs[i]
 * (device) receives the address that holds block i, d_status[i] (device) its status.
 * Blocks until every copy has landed; a set with no evictable way is retried, not
 * reported.  The sticky error is returned. */
#define AGILE_ISSUE_SHARE 0x1u
#define AGILE_BUF_OWNER 1u   /* copied into this request's buffer, registered as the owner */
#define AGILE_BUF_PRIVATE 2u /* copied into this request's buffer, not in the Share Table */
#define AGILE_BUF_SHARED 3u  /* d_ptrs[i] is a live holder's buffer; nothing was copied */
agile_status agile_async_issue(agile_ctx ctx, agile_store store, const uint64_t* d_blocks, uint32_t n,
                               void* const* d_bufs, void** d_ptrs, uint32_t* d_status,
                               uint32_t flags, void* stream);

/* Drops the Share Table holds that agile_async_issue returned: request i's hold of block
 * d_blocks[i] when d_status[i] is AGILE_BUF_OWNER or AGILE_BUF_SHARED (others are
 * skipped).  A block with no holder left is free for a new owner.  Releasing more often
 * than held raises the sticky error (AGILE_ESTATE).  Blocks. */
agile_status agile_buffers_release(agile_ctx ctx, const uint64_t* d_blocks, const uint32_t* d_status,
                                   uint32_t n, void* stream);

/* The owner propagates its buffer's changes to the cache (Sec. 3.4.1): block d_blocks[i]
 * takes the 4096 bytes at d_srcs[i] (device, 16-byte aligned) inside its cache line
 * (the line is read first on a miss; a line being written back is modified once that
 * write has landed), and the line becomes MODIFIED, to be written back on eviction or
 * at agile_flush.  Requests for the same line are applied in turn, lowest index first
 * within a wavefront.  Blocks; returns the sticky error. */
agile_status agile_buffers_writeback(agile_ctx ctx, agile_store store, const uint64_t* d_blocks,
                                     const void* const* d_srcs, uint32_t n, void* stream);

/* Empties the Share Table (every holder forgotten).  For use between phases with no
 * buffer shared.  Blocks. */
agile_status agile_share_reset(agile_ctx ctx);

/* Drops every clean, unpinned line (cold cache).  Dirty lines make it fail with
 * AGILE_ESTATE (flush first).  Blocks until done. */
agile_status agile_invalidate(agile_ctx ctx, agile_store store, void* stream);

/* Blocks until the stream is idle and returns the sticky device error, if any. */
agile_status agile_sync(agile_ctx ctx, void* stream);

/* Counters; see agile_stats.  reset != 0 zeroes them after reading (blocking). */
typedef struct agile_stats {
  uint64_t requests;   /* lookups presented to the cache (a lookup whose prefetched
                          chunk was dropped after an EAGAIN is presented again) */
  uint64_t hits;       /* lookups served by a line resident or in flight at probe time */
  uint64_t misses;     /* lookups whose wavefront issued the READ that filled the line */
  uint64_t read_cmds;  /* READ commands submitted */
  uint64_t write_cmds; /* WRITE commands submitted */
  uint64_t wb_evict;   /* write-backs of dirty victims */
  uint64_t wb_flush;   /* write-backs issued by agile_flush */
  uint64_t eagain;     /* acquisitions that found no evictable way */
  uint64_t sq_spins;   /* submit-loop iterations that made no progress */
  uint64_t ctrl_cmds;  /* commands executed by the emulated controller */
  uint64_t cq_entries; /* completion entries consumed by the completion service */
  uint64_t submitted;  /* commands submitted (monotonic, not reset) */
  uint64_t completed;  /* commands completed (monotonic, not reset) */
  uint64_t consumed;   /* workload rows read out of the cache and used */
  uint64_t rows_updated; /* rows written by the backward pass (one per distinct row) */
} agile_stats;
agile_status agile_get_stats(agile_ctx ctx, agile_stats* out, int reset);

/* Static description of a status code; never NULL. */
const char* agile_status_string(agile_status s);
/* Text of the last error recorded on ctx (host or device side); never NULL. */
const char* agile_last_error(agile_ctx ctx);

/* Information for benches and tests (all host values). */
typedef struct agile_info {
  uint32_t num_lines, num_sets, assoc, line_bytes;
  uint32_t num_qp, qp_depth, ctrl_waves, cq_waves;
  uint32_t cu_count, max_user_waves; /* user wavefronts one launch may run */
  uint64_t wallclock_hz;             /* rate of s_memrealtime */
  uint64_t cache_base;               /* device address of line 0 */
  uint32_t service_lds_bytes;        /* LDS (static + dynamic) per workgroup of an
                                        embedding-bag launch, dim 65..128 */
  uint32_t service_blocks;           /* workgroups that run service wavefronts */
} agile_info;
agile_status agile_get_info(agile_ctx ctx, agile_info* out);

/* Caps the user wavefronts of later workload launches (0 = fill the GPU), e.g. to run
 * the thread-level overlap experiment of Sec. 4.2 on one 1024-thread group.  While a cap
 * is set the embedding-bag and gather calls skip their resident-hit pass, so the cap
 * holds for hits too. */
agile_status agile_set_max_user_waves(agile_ctx ctx, uint32_t n);

/* ---------------------------------------------------------------- workloads --------
 * Tables: `num_tables` fp32 tables of `rows` x `dim`, concatenated row-major in the
 * store image starting at byte `base_offset`.  Row bytes (dim*4) must divide 4096. */
typedef struct agile_tables {
  uint64_t rows;
  uint32_t dim;
  uint32_t num_tables;
  uint64_t base_offset;
} agile_tables;

#define AGILE_MODE_SYNC 0u  /* issue, wait, compute, release per chunk (the plain method) */
#define AGILE_MODE_ASYNC 1u /* reads for the next chunk are issued before this chunk is
                               computed, overlapping I/O with compute (Sec. 4.2) */

/* The array-like synchronous access of Sec. 3.5 (Listing 1, method 3), for a batch:
 * gathers n rows, d_out[i*dim + d] = table[d_idx[i] / rows][d_idx[i] % rows][d], where
 * d_idx holds global row numbers (int64, device) and d_out is device fp32 [n, dim].  Rows
 * go through the cache with the two-level coalescing of Sec. 3.3.2 (duplicates within a
 * wavefront, then the cache).  Stream-ordered; errors as for the workloads below. */
agile_status agile_gather(agile_ctx ctx, agile_store store, const agile_tables* tb,
                          const int64_t* d_idx, uint64_t n, uint32_t mode, float* d_out,
                          void* stream);

/* Embedding-bag forward: B samples x T = num_tables bags in sample-major order; bag
 * g = b*T + t covers lookups [d_off[g], d_off[g+1]) of table t (d_idx: row numbers within
 * the table).  d_out[g*dim + d] = sum, in lookup order, of f_K(row value), where f_K is
 * K iterations of v = fmaf(v, 0.999f, 0.001f) (a compute loop that sets the
 * computation-to-communication ratio, Sec. 4.2); fp32 accumulator from +0.0f.
 * mode is AGILE_MODE_SYNC or AGILE_MODE_ASYNC; both give bit-identical output.
 * Stream-ordered, two kernel launches: a resident-hit pass (one wavefront per bag, no
 * queue traffic) serves the bags whose lines are all cached and defers the others to
 * the I/O launch, which runs them through the cache and queues (with a wave cap from
 * agile_set_max_user_waves only the I/O launch runs, for every bag).  No host
 * synchronisation, allocation or memset: the call may be captured in a HIP graph and the
 * graph replayed, once an eager call with a table of the same dim has been made on the
 * context (it caches an occupancy query). */
agile_status agile_embbag_forward(agile_ctx ctx, agile_store store, const agile_tables* tb,
                                  const int64_t* d_idx, const int64_t* d_off, uint64_t B,
                                  uint32_t K, uint32_t mode, float* d_out, void* stream);

/* The asynchronous mode of Sec. 4.3's DLRM runs: this batch is computed while the next
 * batch's data is prefetched into the cache (Listing 1's prefetch(), Sec. 3.5), so the
 * store works on batch n+1 while the GPU computes batch n.  Computes exactly what
 * agile_embbag_forward computes for (d_idx, d_off, B, K) into d_out (bit-identical, any
 * mode), and requests every line of the next batch (d_next_idx, d_next_off, B_next: the
 * same layout and tables) that is neither resident nor in flight, without pinning it: a
 * set with no evictable way drops the request, a row outside the store is skipped, and a
 * prefetched line may be evicted again before it is used (the next call then reads it on
 * demand; results never depend on the prefetch).  When the call's work on the stream has
 * completed, so have all its prefetch reads.  B_next == 0 prefetches nothing (the call is
 * then agile_embbag_forward in AGILE_MODE_ASYNC); B == 0 only prefetches (d_idx, d_off and
 * d_out may then be NULL).  d_next_idx may be NULL when every next bag is empty.
 * Stream-ordered, one launch: the service wavefronts, 64 prefetch wavefronts that submit
 * the next batch's reads and then compute, and every other wavefront computing this
 * batch's bags, each served from resident lines where it can be and through the cache
 * and queues from where it cannot (the same wave count as the I/O launch of
 * agile_embbag_forward); a launch of at most 256 wavefronts (a small cache, or a cap
 * from agile_set_max_user_waves) has every wavefront prefetch and compute in turns.
 * No host synchronisation, allocation or memset: the call may be captured in a HIP graph
 * and replayed, as agile_embbag_forward.  With AGILE_F_SERIALIZED nothing is prefetched.
 * Errors as for agile_embbag_forward. */
agile_status agile_embbag_forward_prefetch(agile_ctx ctx, agile_store store, const agile_tables* tb,
                                           const int64_t* d_idx, const int64_t* d_off, uint64_t B,
                                           uint32_t K, float* d_out, const int64_t* d_next_idx,
                                           const int64_t* d_next_off, uint64_t B_next, void* stream);

/* ---------------------------------------------------------------- diagnostics ------
 * For tests and tools; not part of the I/O path. */

/* Runs n requests one at a time on one lane (issue, wait, release): request i asks for
 * line id d_lines[i] (uint64) and, when d_writes (uint8, may be NULL) is non-zero, marks
 * the line MODIFIED.  Writes d_hit[i] (1 when no READ was needed) and d_way[i] (the way
 * that served it).  With nothing else running, the sequence of hits, ways and dirty
 * write-backs equals that of a sequential clock cache (Sec. 3.4, Sec. 4.4).  Blocks. */
agile_status agile_debug_trace(agile_ctx ctx, agile_store store, const uint64_t* d_lines,
                               const uint8_t* d_writes, uint64_t n, uint8_t* d_hit,
                               int32_t* d_way, void* stream);

/* Roofline probe (measurement only): `waves` wavefronts copy n 4 KiB blocks from src
 * (pinned host memory or device memory) into d_dst (device, dst_blocks blocks), block i
 * being src block d_list[i] (device uint64; NULL = i), `per_wave` (1..4) blocks in flight
 * per wave, with the emulated controller's copy routine.  Stream-ordered. */
agile_status agile_probe_copy(const void* src, const uint64_t* d_list, uint64_t n, void* d_dst,
                              uint64_t dst_blocks, uint32_t waves, uint32_t per_wave,
                              void* stream);

/* The library's own device-wide exclusive prefix sum (used per BFS level):
 * d_out[i] = d_in[0] + ... + d_in[i-1] (uint64, device; d_out may equal d_in).  Allocates
 * its work area; blocks. */
agile_status agile_debug_exclusive_scan_u64(const uint64_t* d_in, uint64_t* d_out, uint64_t n,
                                            void* stream);

/* The library's own stable LSD radix sort (used by the backward pass): sorts the n
 * uint64 keys of d_keys (device, in place) by their bits [lo, hi), keeping the input
 * order of keys whose bits agree.  Allocates its work area; blocks. */
agile_status agile_debug_radix_sort_u64(uint64_t* d_keys, uint64_t n, uint32_t lo, uint32_t hi,
                                        void* stream);

/* The lock-chain walker of AGILE_F_LOCKCHAIN run on a given wait state (diagnostics):
 * waits[w] (host, n_waits entries) is what wave w waits for, encoded as the walker
 * records it (kind << 56 | object: kind 0x0A = the set lock of store line `object`,
 * 0x0D = the fill of cache line `object`, 0x0B its write-back, 0x01 an SQ slot
 * (q << 32 | ticket), 0x0F a free way; 0 = not waiting); set lock_sets[i] (host) is given
 * the word lock_words[i] (holder wave + 2, or 1 for an unnamed holder).  The walk starts
 * at wave start_wave waiting for start_what; the chain's text goes to msg (host,
 * msg_len bytes, NUL-terminated).  The state is cleared afterwards (waits, the given set
 * locks, the chain).  No other call may run on the context meanwhile.  Blocks. */
agile_status agile_debug_lockchain(agile_ctx ctx, const uint64_t* waits, uint32_t n_waits,
                                   const uint32_t* lock_sets, const uint32_t* lock_words,
                                   uint32_t n_locks, uint32_t start_wave, uint64_t start_what,
                                   char* msg, uint32_t msg_len);

/* Raw device counters in their internal order (for diagnostics): out[i] for i < n. */
agile_status agile_debug_counters(agile_ctx ctx, uint64_t* out, uint32_t n);

/* Decodes every line's metadata into device arrays: tag (int64, -1 when INVALID), state
 * (uint8: 0 INVALID, 1 FETCHING, 2 READY, 3 DIRTY, 4 WRITEBACK) and pin count (uint32).
 * Blocks. */
agile_status agile_debug_dump(agile_ctx ctx, int64_t* d_tags, uint8_t* d_states,
                              uint32_t* d_rc, void* stream);

/* Embedding-bag backward fused with SGD, for the loss L = sum_g sum_d grad[g][d] *
 * pooled[g][d] of agile_embbag_forward with K = 0: for every distinct row r of table t
 * looked up by the batch, g = the sum of d_grad[bag] over the row's occurrences in
 * ascending lookup position (fp32 from +0.0f), then w = fmaf(-lr, g, w) is applied to the
 * row inside its HBM cache line, which becomes MODIFIED (Sec. 3.4) and is written back to
 * the store when evicted or at agile_flush.  n is the total number of lookups
 * (d_off[B*T]); d_grad is [B*T, dim] fp32 (device).  Stream-ordered; uses a work area the
 * context grows on demand. */
agile_status agile_embbag_backward_sgd(agile_ctx ctx, agile_store store, const agile_tables* tb,
                                       const int64_t* d_idx, const int64_t* d_off, uint64_t B,
                                       uint64_t n, const float* d_grad, float lr, void* stream);

/* agile_embbag_backward_sgd of this batch while the next batch (d_next_idx, d_next_off,
 * B_next: the layout of agile_embbag_forward, same tables) is prefetched into the cache,
 * as agile_embbag_forward_prefetch does it (Sec. 4.3's asynchronous mode, here for a
 * training step: the next step's forward then finds its lines resident; Listing 1's
 * prefetch()).  The updates are exactly those of agile_embbag_backward_sgd.  The
 * prefetch is unpinned and best effort: a line whose set has no evictable way is not
 * fetched, and a prefetched line may be evicted again (a DIRTY victim is written back
 * first).  Stream-ordered, one launch for the updates (its leading 64 wavefronts first
 * prefetch, with at most a bounded number of commands in flight, then update rows);
 * B_next == 0 is agile_embbag_backward_sgd; n == 0 only prefetches.  Uses the work area
 * of agile_embbag_backward_sgd; errors as for it. */
agile_status agile_embbag_backward_sgd_prefetch(agile_ctx ctx, agile_store store, const agile_tables* tb,
                                                const int64_t* d_idx, const int64_t* d_off, uint64_t B,
                                                uint64_t n, const float* d_grad, float lr,
                                                const int64_t* d_next_idx, const int64_t* d_next_off,
                                                uint64_t B_next, void* stream);

/* The same backward pass for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): identical
 * arguments, results and errors, but the work area (sort keys, bag ids, row heads,
 * counters, the radix sort's buffers: about 25 MiB) is one fixed array in device memory
 * that the library holds on each device from agile_init until the process ends, instead
 * of the context's growable area.  n (lookups) must be <= 1,048,576 (2^20); a larger n is
 * rejected with AGILE_EINVAL before anything is launched.  No call allocates or frees
 * memory.  Every call on one device shares that array, and each call leaves its contents
 * behind (the counters are cleared by the call itself): calls that overlap in time on one
 * device, from any context or stream, race and must not be issued. */
agile_status agile_embbag_backward_sgd_noalloc(agile_ctx ctx, agile_store store,
                                               const agile_tables* tb, const int64_t* d_idx,
                                               const int64_t* d_off, uint64_t B, uint64_t n,
                                               const float* d_grad, float lr, void* stream);

/* A CSR graph held in the store: row_ptr int64[V+1] at row_ptr_offset, col int32[E] at
 * col_offset and, for SpMV, val fp32[E] at val_offset (byte offsets into the store). */
typedef struct agile_csr {
  uint64_t num_vertices;
  uint64_t num_edges;
  uint64_t row_ptr_offset;
  uint64_t col_offset;
  uint64_t val_offset;
} agile_csr;

/* Level-synchronous top-down BFS over out-edges (the graph application of Sec. 4.5,
 * without application-level optimisation): d_level (int32[V], device) receives the hop
 * distance from src, -1 when unreached.  row_ptr and col are read through the cache.
 * Blocks (one host step per level); *out_levels (may be NULL) receives the number of
 * levels including the source's. */
agile_status agile_bfs(agile_ctx ctx, agile_store store, const agile_csr* g, uint64_t src,
                       int32_t* d_level, uint32_t* out_levels, void* stream);

/* CSR SpMV (Sec. 4.5): d_y[i] = fold over k ascending in row i of
 * acc = fmaf(val[k], d_x[col[k]], acc), acc from +0.0f.  row_ptr, col and val are read
 * through the cache; d_x and d_y are device fp32[V].  Stream-ordered. */
agile_status agile_spmv(agile_ctx ctx, agile_store store, const agile_csr* g, const float* d_x,
                        float* d_y, void* stream);

/* The kernel-only baselines of the breakdown in Sec. 4.5: the same BFS and SpMV kernels
 * (same levels, same fold order, so bit-identical results) reading a copy of the store
 * image resident in device memory (d_image, image_bytes, the same layout and offsets)
 * with no cache, queue or service wavefront involved.  The context supplies the launch
 * geometry and the work area; no store needs to be open.  Blocking as agile_bfs /
 * stream-ordered as agile_spmv. */
agile_status agile_bfs_resident(agile_ctx ctx, const void* d_image, uint64_t image_bytes,
                                const agile_csr* g, uint64_t src, int32_t* d_level,
                                uint32_t* out_levels, void* stream);
agile_status agile_spmv_resident(agile_ctx ctx, const void* d_image, uint64_t image_bytes,
                                 const agile_csr* g, const float* d_x, float* d_y, void* stream);

/* The same kernel-only baseline for the embedding-bag forward (Sec. 4.4's DLRM lookups):
 * the tables read straight from a copy of the store image resident in device memory
 * (d_image, image_bytes; tb, d_idx, d_off, B, K and d_out as in agile_embbag_forward),
 * with no cache, queue or service wavefront; the outputs are bit-identical to the cached
 * forward's.  A row index outside [0, rows) contributes nothing and raises the sticky
 * error (AGILE_ESTATE from the next blocking call).  No store needs to be open.
 * Stream-ordered. */
agile_status agile_embbag_forward_resident(agile_ctx ctx, const void* d_image, uint64_t image_bytes,
                                           const agile_tables* tb, const int64_t* d_idx,
                                           const int64_t* d_off, uint64_t B, uint32_t K,
                                           float* d_out, void* stream);

/* ---------------------------------------------------------------- serving --------- */
typedef struct agile_serve_opts {
  uint64_t max_inflight_lookups;  /* queue budget (0 = the SQ slots, or the largest request) */
  uint64_t max_inflight_requests; /* 0 = 4096 */
  uint64_t user_waves;            /* 0 = num_lines / 16; else this many (up to what fits) */
  uint64_t max_inflight_lines;    /* cache budget (0 = num_lines); a request reserves
                                     min(its lookups, 64, budget / 2) lines */
} agile_serve_opts;

typedef struct agile_serve_report {
  double elapsed_s;
  uint64_t requests, bags, lookups;
  uint64_t max_inflight_requests;
  uint64_t user_waves;
} agile_serve_report;

/* Serving session (embedding-bag lookups; Sec. 3.2's asynchronous, GPU-initiated reads
 * applied to requests that arrive while the kernel runs).  agile_session_open launches
 * one persistent kernel on a stream of its own; its wavefronts claim bags in submission
 * order, wait for a bag until the host has published it, and run it through the cache
 * and queues as agile_embbag_forward does, so the bags of requests submitted while
 * others are on the GPU are picked up as waves free up and their I/O overlaps on the
 * device.  While a session is open the context accepts no other call (AGILE_ESTATE)
 * except the session calls, agile_get_info, agile_last_error and agile_shutdown (which
 * closes the session first).  One session per context at a time.
 *
 * Requests travel through rings in pinned host memory that the session owns: the host
 * writes a request's bag descriptors and lookups into the next free slots, then
 * publishes the new count of bags with a release store; one service wavefront of the
 * kernel copies each published batch into HBM copies of the rings before the other
 * wavefronts see it; the kernel writes each bag's output into the bag's ring slot (host
 * memory) and raises the request's done flag (system scope) after its last bag.  Slots
 * are reused in submission order once requests are polled.
 *
 * tb, K, mode: as agile_embbag_forward (dim <= 256, 4096 % (4*dim) == 0).
 * opts: admission budgets and the wave count (NULL = defaults, see agile_serve_opts).
 * Returns AGILE_ENOMEM when the rings cannot be allocated. */
typedef struct agile_session_s* agile_session;
agile_status agile_session_open(agile_ctx ctx, agile_store store, const agile_tables* tb, uint32_t K,
                                uint32_t mode, const agile_serve_opts* opts, agile_session* out);

/* Submits one request of nbags bags (1 <= nbags, and at most 65,536 lookups and bags):
 * bag k owns lookups [bag_off[k], bag_off[k+1]) of idx (host memory, bag_off[0] == 0,
 * non-decreasing; rows in [0, rows)) and reads table k % num_tables.  The caller's
 * arrays are copied before the call returns.  *out_req receives the request's number
 * (0, 1, 2, ... in submission order).  AGILE_EAGAIN: the requests in flight leave no
 * room in a budget (queue: lookups in flight; cache: the lines one chunk of each
 * request can pin, min(lookups, 64, budget / 2); requests in flight) or in a ring; poll
 * and retry.  A request is always admitted when none is in flight. */
agile_status agile_session_submit(agile_session s, uint32_t nbags, const int64_t* bag_off,
                                  const int64_t* idx, uint64_t* out_req);

/* Non-blocking: AGILE_OK once request req has completed, with its nbags*dim pooled
 * outputs copied to out (host memory; NULL discards them); AGILE_EAGAIN while it runs.
 * Each request is collected once (AGILE_EINVAL after that, or for an unknown number).
 * AGILE_ETIMEDOUT if the kernel was aborted (the context is then poisoned). */
agile_status agile_session_poll(agile_session s, uint64_t req, float* out);

/* Waits for every submitted request to complete (outputs not yet polled are dropped),
 * stops the kernel, frees the rings and releases the context.  The handle is invalid
 * afterwards.  AGILE_ETIMEDOUT when requests do not complete within the watchdog. */
agile_status agile_session_close(agile_session s);

/* Replay harness, a client of the session calls above: it submits request r once
 * arrival_s[r] (seconds from the start, non-decreasing) has passed and the session
 * admits it (a request that does not fit waits, and so do the ones behind it), polls
 * the requests in flight, and closes the session at the end.  Request r owns bags
 * [req_bag0[r], req_bag0[r+1]); bag b owns lookups [bag_off[b], bag_off[b+1]) of idx and
 * reads table (b - req_bag0[r]) % num_tables.  Outputs (pooled, K as in
 * agile_embbag_forward) go to out[b*dim ...]; latency_s[r] is the time from arrival to
 * the host seeing request r's outputs in host memory.  All arrays are host memory;
 * blocks for the whole session. */
agile_status agile_serve(agile_ctx ctx, agile_store store, const agile_tables* tb, uint32_t K,
                         uint32_t mode, uint64_t nreq, const double* arrival_s,
                         const int64_t* req_bag0, const int64_t* bag_off, const int64_t* idx,
                         float* out, double* latency_s, const agile_serve_opts* opts,
                         agile_serve_report* report);

#ifdef __cplusplus
}
#endif
#endif /* AGILE_H */
