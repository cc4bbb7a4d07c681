"""Python binding of libagile.so (include/agile.h): argument marshalling only.

Every step of the path runs in the library's HIP kernels; this module only converts
torch tensors / numpy arrays into pointers and checks status codes.  It raises loudly
when the native library is missing: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libagile.so")

OK, EINVAL, ENOMEM, EHIP, ETIMEDOUT, EAGAIN, EIO, EPROTO, ESTATE = 0, -1, -2, -3, -4, -5, -6, -7, -8
F_SERIALIZED, F_NO_PRIO, F_PROFILE, F_LOCKCHAIN = 0x1, 0x2, 0x4, 0x8
MODE_SYNC, MODE_ASYNC = 0, 1


class AgileError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class Config(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("device", C.c_int32), ("cache_bytes", C.c_uint64),
                ("line_bytes", C.c_uint32), ("assoc", C.c_uint32), ("num_qp", C.c_uint32),
                ("qp_depth", C.c_uint32), ("ctrl_waves", C.c_uint32), ("cq_waves", C.c_uint32),
                ("max_user_waves", C.c_uint32), ("latency_ns", C.c_uint64),
                ("iops_cap", C.c_uint64), ("timeout_ns", C.c_uint64), ("flags", C.c_uint32),
                ("reserved", C.c_uint32)]


class Stats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in (
        "requests", "hits", "misses", "read_cmds", "write_cmds", "wb_evict", "wb_flush",
        "eagain", "sq_spins", "ctrl_cmds", "cq_entries", "submitted", "completed",
        "consumed", "rows_updated")]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


class Info(C.Structure):
    _fields_ = [("num_lines", C.c_uint32), ("num_sets", C.c_uint32), ("assoc", C.c_uint32),
                ("line_bytes", C.c_uint32), ("num_qp", C.c_uint32), ("qp_depth", C.c_uint32),
                ("ctrl_waves", C.c_uint32), ("cq_waves", C.c_uint32), ("cu_count", C.c_uint32),
                ("max_user_waves", C.c_uint32), ("wallclock_hz", C.c_uint64),
                ("cache_base", C.c_uint64), ("service_lds_bytes", C.c_uint32),
                ("service_blocks", C.c_uint32)]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


class CSR(C.Structure):
    _fields_ = [("num_vertices", C.c_uint64), ("num_edges", C.c_uint64),
                ("row_ptr_offset", C.c_uint64), ("col_offset", C.c_uint64),
                ("val_offset", C.c_uint64)]


class ServeOpts(C.Structure):
    _fields_ = [("max_inflight_lookups", C.c_uint64), ("max_inflight_requests", C.c_uint64),
                ("user_waves", C.c_uint64), ("max_inflight_lines", C.c_uint64)]


class ServeReport(C.Structure):
    _fields_ = [("elapsed_s", C.c_double), ("requests", C.c_uint64), ("bags", C.c_uint64),
                ("lookups", C.c_uint64), ("max_inflight_requests", C.c_uint64),
                ("user_waves", C.c_uint64)]

    def as_dict(self):
        return {n: (float(getattr(self, n)) if n == "elapsed_s" else int(getattr(self, n)))
                for n, _ in self._fields_}


class Tables(C.Structure):
    _fields_ = [("rows", C.c_uint64), ("dim", C.c_uint32), ("num_tables", C.c_uint32),
                ("base_offset", C.c_uint64)]


_lib = None


def lib():
    """Loads libagile.so; raises if it is not built (no CPU fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build()")
        # torch ships its own HIP runtime under the same soname; loading torch first makes
        # this library bind to that one instance instead of a second runtime
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        vp, u32, u64, i32, st = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int32, C.c_int
        sig = {
            "agile_config_default": (None, [C.POINTER(Config)]),
            "agile_init": (st, [C.POINTER(Config), C.POINTER(vp)]),
            "agile_shutdown": (st, [vp]),
            "agile_host_alloc": (st, [u64, C.POINTER(vp)]),
            "agile_host_free": (st, [vp]),
            "agile_open_store": (st, [vp, vp, u64, u32, u32, C.POINTER(vp)]),
            "agile_close_store": (st, [vp, vp]),
            "agile_async_read": (st, [vp, vp, vp, u32, vp, vp]),
            "agile_wait": (st, [vp, vp, u32, vp, vp]),
            "agile_release": (st, [vp, vp, u32, vp]),
            "agile_flush": (st, [vp, vp, vp]),
            "agile_invalidate": (st, [vp, vp, vp]),
            "agile_sync": (st, [vp, vp]),
            "agile_get_stats": (st, [vp, C.POINTER(Stats), C.c_int]),
            "agile_status_string": (C.c_char_p, [st]),
            "agile_last_error": (C.c_char_p, [vp]),
            "agile_get_info": (st, [vp, C.POINTER(Info)]),
            "agile_set_max_user_waves": (st, [vp, u32]),
            "agile_gather": (st, [vp, vp, C.POINTER(Tables), vp, u64, u32, vp, vp]),
            "agile_embbag_forward": (st, [vp, vp, C.POINTER(Tables), vp, vp, u64, u32, u32, vp,
                                          vp]),
            "agile_embbag_forward_prefetch": (st, [vp, vp, C.POINTER(Tables), vp, vp, u64, u32,
                                                   vp, vp, vp, u64, vp]),
            "agile_debug_trace": (st, [vp, vp, vp, vp, u64, vp, vp, vp]),
            "agile_embbag_backward_sgd": (st, [vp, vp, C.POINTER(Tables), vp, vp, u64, u64, vp,
                                               C.c_float, vp]),
            "agile_embbag_backward_sgd_prefetch": (st, [vp, vp, C.POINTER(Tables), vp, vp, u64,
                                                        u64, vp, C.c_float, vp, vp, u64, vp]),
            "agile_debug_dump": (st, [vp, vp, vp, vp, vp]),
            "agile_debug_counters": (st, [vp, vp, u32]),
            "agile_probe_copy": (st, [vp, vp, u64, vp, u64, u32, u32, vp]),
            "agile_bfs": (st, [vp, vp, C.POINTER(CSR), u64, vp, C.POINTER(C.c_uint32), vp]),
            "agile_spmv": (st, [vp, vp, C.POINTER(CSR), vp, vp, vp]),
            "agile_serve": (st, [vp, vp, C.POINTER(Tables), u32, u32, u64, vp, vp, vp, vp, vp,
                                 vp, C.POINTER(ServeOpts), C.POINTER(ServeReport)]),
            "agile_debug_exclusive_scan_u64": (st, [vp, vp, u64, vp]),
            "agile_bfs_resident": (st, [vp, vp, u64, C.POINTER(CSR), u64, vp, C.POINTER(C.c_uint32),
                                        vp]),
            "agile_spmv_resident": (st, [vp, vp, u64, C.POINTER(CSR), vp, vp, vp]),
            "agile_embbag_backward_sgd_noalloc": (st, [vp, vp, C.POINTER(Tables), vp, vp, u64, u64,
                                                       vp, C.c_float, vp]),
            "agile_debug_radix_sort_u64": (st, [vp, u64, u32, u32, vp]),
            "agile_session_open": (st, [vp, vp, C.POINTER(Tables), u32, u32, C.POINTER(ServeOpts),
                                        C.POINTER(vp)]),
            "agile_session_submit": (st, [vp, u32, vp, vp, C.POINTER(C.c_uint64)]),
            "agile_session_poll": (st, [vp, u64, vp]),
            "agile_session_close": (st, [vp]),
            "agile_open_store_striped": (st, [vp, C.POINTER(vp), u32, u64, u32, u32,
                                              C.POINTER(vp)]),
            "agile_write": (st, [vp, vp, vp, u32, vp, vp]),
            "agile_embbag_forward_resident": (st, [vp, vp, u64, C.POINTER(Tables), vp, vp, u64, u32,
                                                   vp, vp]),
            "agile_debug_lockchain": (st, [vp, vp, u32, vp, vp, u32, u32, u64, C.c_char_p, u32]),
            "agile_async_issue": (st, [vp, vp, vp, u32, vp, vp, vp, u32, vp]),
            "agile_buffers_release": (st, [vp, vp, vp, u32, vp]),
            "agile_buffers_writeback": (st, [vp, vp, vp, vp, u32, vp]),
            "agile_share_reset": (st, [vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def status_string(s: int) -> str:
    return lib().agile_status_string(s).decode()


def _ptr(x) -> int:
    """Device or host address of a torch tensor, numpy array or int."""
    if x is None:
        return 0
    if isinstance(x, int):
        return x
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    return x.data_ptr()


def _stream(stream) -> int:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def probe_copy(src, lst, n: int, dst, dst_blocks: int, waves: int, per_wave: int, stream=None):
    """Roofline probe: copies n 4 KiB blocks (see agile_probe_copy)."""
    s = lib().agile_probe_copy(_ptr(src), _ptr(lst), n, _ptr(dst), dst_blocks, waves, per_wave,
                               _stream(stream))
    if s != OK:
        raise AgileError(s, "agile_probe_copy")


def exclusive_scan_u64(d_in, d_out, n: int, stream=None):
    """The library's device-wide exclusive prefix sum (agile_debug_exclusive_scan_u64)."""
    s = lib().agile_debug_exclusive_scan_u64(_ptr(d_in), _ptr(d_out), n, _stream(stream))
    if s != OK:
        raise AgileError(s, "agile_debug_exclusive_scan_u64")


def radix_sort_u64(d_keys, n: int, lo: int, hi: int, stream=None):
    """The library's stable radix sort by bits [lo, hi) (agile_debug_radix_sort_u64)."""
    s = lib().agile_debug_radix_sort_u64(_ptr(d_keys), n, lo, hi, _stream(stream))
    if s != OK:
        raise AgileError(s, "agile_debug_radix_sort_u64")


def default_config(**kw) -> Config:
    cfg = Config()
    lib().agile_config_default(C.byref(cfg))
    for k, v in kw.items():
        if not hasattr(cfg, k):
            raise TypeError(f"unknown config field {k}")
        setattr(cfg, k, v)
    return cfg


class PinnedBuffer:
    """Pinned, device-mapped host memory (agile_host_alloc) with a numpy view."""

    def __init__(self, nbytes: int):
        p = C.c_void_p()
        s = lib().agile_host_alloc(nbytes, C.byref(p))
        if s != OK:
            raise AgileError(s, f"agile_host_alloc({nbytes})")
        self.ptr = p.value
        self.nbytes = nbytes
        self.array = np.ctypeslib.as_array((C.c_uint8 * nbytes).from_address(self.ptr))

    def free(self):
        if self.ptr:
            lib().agile_host_free(self.ptr)
            self.ptr = 0
            self.array = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Store:
    def __init__(self, ctx: "Context", handle: int, image: PinnedBuffer | None, nbytes: int):
        self.ctx, self.handle, self.image, self.nbytes = ctx, handle, image, nbytes


class Session:
    """An open serving session: submit requests, poll for their outputs, close."""

    def __init__(self, ctx: "Context", h: int, dim: int):
        self.ctx, self.h, self.dim = ctx, h, dim

    def submit(self, bag_off, idx):
        """Submits one request (bag k = lookups [bag_off[k], bag_off[k+1]) of idx).
        Returns its number, or None when the session has no room for it yet."""
        bag_off = np.ascontiguousarray(bag_off, dtype=np.int64)
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        r = C.c_uint64()
        s = lib().agile_session_submit(self.h, bag_off.size - 1, _ptr(bag_off),
                                       _ptr(idx) if idx.size else 0, C.byref(r))
        if s == EAGAIN:
            return None
        self.ctx._check(s, "agile_session_submit")
        return int(r.value)

    def poll(self, req: int, nbags: int):
        """The [nbags, dim] outputs of request req once it has completed, else None."""
        out = np.empty((nbags, self.dim), dtype=np.float32)
        s = lib().agile_session_poll(self.h, req, _ptr(out))
        if s == EAGAIN:
            return None
        self.ctx._check(s, "agile_session_poll")
        return out

    def close(self):
        if self.h:
            h, self.h = self.h, None
            self.ctx._check(lib().agile_session_close(h), "agile_session_close")

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Context:
    def __init__(self, cfg: Config | None = None, **kw):
        cfg = cfg if cfg is not None else default_config(**kw)
        self.cfg = cfg
        h = C.c_void_p()
        s = lib().agile_init(C.byref(cfg), C.byref(h))
        if s != OK:
            raise AgileError(s, "agile_init")
        self.h = h.value
        self.store = None

    # ---- helpers
    def _check(self, s: int, what: str):
        if s != OK:
            msg = f"{what}: {lib().agile_last_error(self.h).decode()}"
            if s in (ETIMEDOUT, EPROTO, EIO):
                try:
                    msg += f" counters={self.debug_counters()}"
                except Exception:
                    pass
            raise AgileError(s, msg)

    def last_error(self) -> str:
        return lib().agile_last_error(self.h).decode()

    # ---- lifecycle
    def open_store(self, image: PinnedBuffer | int, nbytes: int | None = None) -> Store:
        ptr = image.ptr if isinstance(image, PinnedBuffer) else int(image)
        nbytes = nbytes if nbytes is not None else image.nbytes
        h = C.c_void_p()
        self._check(lib().agile_open_store(self.h, ptr, nbytes, 4096, 0, C.byref(h)),
                    "agile_open_store")
        self.store = Store(self, h.value, image if isinstance(image, PinnedBuffer) else None,
                           nbytes)
        return self.store

    def open_store_striped(self, images, nbytes_each: int | None = None) -> Store:
        """A store striped line by line over several emulated devices, one image each
        (agile_open_store_striped): store line l is line l // n of images[l % n]."""
        ptrs = [im.ptr if isinstance(im, PinnedBuffer) else int(im) for im in images]
        if nbytes_each is None:
            nbytes_each = images[0].nbytes
        arr = (C.c_void_p * len(ptrs))(*ptrs)
        h = C.c_void_p()
        self._check(lib().agile_open_store_striped(self.h, arr, len(ptrs), nbytes_each, 4096, 0,
                                                   C.byref(h)), "agile_open_store_striped")
        self.store = Store(self, h.value, None, nbytes_each * len(ptrs))
        self.store.images = list(images)
        return self.store

    def write(self, lines, src, stream=None, store=None):
        """Write-through of whole lines (agile_write): lines[i] gets src[i] (line_bytes)."""
        store = store or self.store
        self._check(lib().agile_write(self.h, store.handle, _ptr(lines), lines.numel(), _ptr(src),
                                      _stream(stream)), "agile_write")

    def close_store(self, store: Store | None = None) -> int:
        store = store or self.store
        s = lib().agile_close_store(self.h, store.handle)
        if s != ESTATE:  # (ESTATE: a serving session is open; the store stays open)
            self.store = None
        return s

    def shutdown(self):
        if self.h:
            lib().agile_shutdown(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.shutdown()

    # ---- ticket API
    def async_read(self, blocks, tickets, stream=None, store=None):
        store = store or self.store
        self._check(lib().agile_async_read(self.h, store.handle, _ptr(blocks), blocks.numel(),
                                           _ptr(tickets), _stream(stream)), "agile_async_read")

    def wait(self, tickets, ptrs, stream=None) -> int:
        s = lib().agile_wait(self.h, _ptr(tickets), tickets.numel(), _ptr(ptrs), _stream(stream))
        if s not in (OK, EAGAIN):
            self._check(s, "agile_wait")
        return s

    def release(self, tickets, stream=None):
        self._check(lib().agile_release(self.h, _ptr(tickets), tickets.numel(), _stream(stream)),
                    "agile_release")

    ISSUE_SHARE = 0x1
    BUF_OWNER, BUF_PRIVATE, BUF_SHARED = 1, 2, 3

    def async_issue(self, blocks, bufs, ptrs, status, share: bool = False, stream=None,
                    store=None):
        """Reads into user buffers (agile_async_issue): bufs/ptrs are device int64 arrays
        of addresses, status a device int32 array."""
        store = store or self.store
        self._check(lib().agile_async_issue(self.h, store.handle, _ptr(blocks), blocks.numel(),
                                            _ptr(bufs), _ptr(ptrs), _ptr(status),
                                            self.ISSUE_SHARE if share else 0, _stream(stream)),
                    "agile_async_issue")

    def buffers_release(self, blocks, status, stream=None):
        self._check(lib().agile_buffers_release(self.h, _ptr(blocks), _ptr(status), blocks.numel(),
                                                _stream(stream)), "agile_buffers_release")

    def buffers_writeback(self, blocks, srcs, stream=None, store=None):
        store = store or self.store
        self._check(lib().agile_buffers_writeback(self.h, store.handle, _ptr(blocks), _ptr(srcs),
                                                  blocks.numel(), _stream(stream)),
                    "agile_buffers_writeback")

    def share_reset(self):
        self._check(lib().agile_share_reset(self.h), "agile_share_reset")

    def flush(self, stream=None, store=None):
        store = store or self.store
        self._check(lib().agile_flush(self.h, store.handle, _stream(stream)), "agile_flush")

    def invalidate(self, stream=None, store=None):
        store = store or self.store
        self._check(lib().agile_invalidate(self.h, store.handle, _stream(stream)),
                    "agile_invalidate")

    def sync(self, stream=None):
        self._check(lib().agile_sync(self.h, _stream(stream)), "agile_sync")

    def stats(self, reset: bool = False) -> dict:
        st = Stats()
        self._check(lib().agile_get_stats(self.h, C.byref(st), 1 if reset else 0),
                    "agile_get_stats")
        return st.as_dict()

    def set_max_user_waves(self, n: int):
        self._check(lib().agile_set_max_user_waves(self.h, n), "agile_set_max_user_waves")

    def info(self) -> dict:
        inf = Info()
        self._check(lib().agile_get_info(self.h, C.byref(inf)), "agile_get_info")
        return inf.as_dict()

    # ---- workloads
    @staticmethod
    def tables(rows: int, dim: int, num_tables: int = 1, base_offset: int = 0) -> Tables:
        return Tables(rows, dim, num_tables, base_offset)

    def gather(self, tb: Tables, idx, out, mode: int = MODE_SYNC, stream=None, store=None):
        store = store or self.store
        self._check(lib().agile_gather(self.h, store.handle, C.byref(tb), _ptr(idx), idx.numel(),
                                       mode, _ptr(out), _stream(stream)), "agile_gather")

    def embbag_forward(self, tb: Tables, idx, off, B: int, K: int, out, mode: int = MODE_SYNC,
                       stream=None, store=None):
        store = store or self.store
        self._check(lib().agile_embbag_forward(self.h, store.handle, C.byref(tb), _ptr(idx),
                                               _ptr(off), B, K, mode, _ptr(out), _stream(stream)),
                    "agile_embbag_forward")

    def embbag_forward_prefetch(self, tb: Tables, idx, off, B: int, K: int, out, next_idx,
                                next_off, B_next: int, stream=None, store=None):
        """Computes this batch (as embbag_forward) while the lines of the next batch
        (next_idx, next_off, B_next samples) are prefetched into the cache, unpinned."""
        store = store or self.store
        self._check(lib().agile_embbag_forward_prefetch(
            self.h, store.handle, C.byref(tb), _ptr(idx), _ptr(off), B, K, _ptr(out),
            _ptr(next_idx), _ptr(next_off), B_next, _stream(stream)),
            "agile_embbag_forward_prefetch")

    def embbag_backward_sgd(self, tb: Tables, idx, off, B: int, grad, lr: float, stream=None,
                            store=None):
        store = store or self.store
        self._check(lib().agile_embbag_backward_sgd(self.h, store.handle, C.byref(tb), _ptr(idx),
                                                    _ptr(off), B, idx.numel(), _ptr(grad), lr,
                                                    _stream(stream)),
                    "agile_embbag_backward_sgd")

    def embbag_backward_sgd_prefetch(self, tb: Tables, idx, off, B: int, grad, lr: float, next_idx,
                                     next_off, B_next: int, stream=None, store=None):
        """The backward with SGD of this batch while the next batch's lines are prefetched."""
        store = store or self.store
        self._check(lib().agile_embbag_backward_sgd_prefetch(
            self.h, store.handle, C.byref(tb), _ptr(idx), _ptr(off), B,
            0 if idx is None else idx.numel(), _ptr(grad), lr,
            _ptr(next_idx), _ptr(next_off), B_next, _stream(stream)),
            "agile_embbag_backward_sgd_prefetch")

    def bfs(self, g: CSR, src: int, level, stream=None, store=None) -> int:
        store = store or self.store
        nl = C.c_uint32(0)
        self._check(lib().agile_bfs(self.h, store.handle, C.byref(g), src, _ptr(level),
                                    C.byref(nl), _stream(stream)), "agile_bfs")
        return int(nl.value)

    def spmv(self, g: CSR, x, y, stream=None, store=None):
        store = store or self.store
        self._check(lib().agile_spmv(self.h, store.handle, C.byref(g), _ptr(x), _ptr(y),
                                     _stream(stream)), "agile_spmv")

    def bfs_resident(self, image, nbytes: int, g: CSR, src: int, level, stream=None) -> int:
        """BFS over a copy of the store image resident in device memory (no cache)."""
        nl = C.c_uint32(0)
        self._check(lib().agile_bfs_resident(self.h, _ptr(image), nbytes, C.byref(g), src,
                                             _ptr(level), C.byref(nl), _stream(stream)),
                    "agile_bfs_resident")
        return int(nl.value)

    def embbag_forward_resident(self, image, nbytes: int, tb: Tables, idx, off, B: int, K: int,
                                out, stream=None):
        """Embedding-bag forward over a copy of the tables resident in device memory (no
        cache); bit-identical to embbag_forward."""
        self._check(lib().agile_embbag_forward_resident(self.h, _ptr(image), nbytes, C.byref(tb),
                                                        _ptr(idx), _ptr(off), B, K, _ptr(out),
                                                        _stream(stream)),
                    "agile_embbag_forward_resident")

    def spmv_resident(self, image, nbytes: int, g: CSR, x, y, stream=None):
        """SpMV over a copy of the store image resident in device memory (no cache)."""
        self._check(lib().agile_spmv_resident(self.h, _ptr(image), nbytes, C.byref(g), _ptr(x),
                                              _ptr(y), _stream(stream)), "agile_spmv_resident")

    def serve(self, tb: Tables, K: int, arrival, req_bag0, bag_off, idx,
              mode: int = MODE_ASYNC, max_inflight_lookups: int = 0,
              max_inflight_requests: int = 0, user_waves: int = 0,
              max_inflight_lines: int = 0, store=None):
        """Continuous-batching session; returns (out [nbags, dim], latency_s, report)."""
        store = store or self.store
        arrival = np.ascontiguousarray(arrival, dtype=np.float64)
        req_bag0 = np.ascontiguousarray(req_bag0, dtype=np.int64)
        bag_off = np.ascontiguousarray(bag_off, dtype=np.int64)
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        nreq = arrival.size
        nbags = int(req_bag0[-1])
        out = np.empty((nbags, tb.dim), dtype=np.float32)
        lat = np.zeros(nreq, dtype=np.float64)
        opts = ServeOpts(max_inflight_lookups, max_inflight_requests, user_waves,
                         max_inflight_lines)
        rep = ServeReport()
        self._check(lib().agile_serve(self.h, store.handle, C.byref(tb), K, mode, nreq,
                                      _ptr(arrival), _ptr(req_bag0), _ptr(bag_off),
                                      _ptr(idx) if idx.size else 0, _ptr(out), _ptr(lat),
                                      C.byref(opts), C.byref(rep)), "agile_serve")
        return out, lat, rep.as_dict()

    def open_session(self, tb: Tables, K: int, mode: int = MODE_ASYNC,
                     max_inflight_lookups: int = 0, max_inflight_requests: int = 0,
                     user_waves: int = 0, max_inflight_lines: int = 0, store=None) -> "Session":
        """Starts a serving session (agile_session_open): a persistent kernel that takes
        requests as they are submitted."""
        store = store or self.store
        opts = ServeOpts(max_inflight_lookups, max_inflight_requests, user_waves,
                         max_inflight_lines)
        h = C.c_void_p()
        self._check(lib().agile_session_open(self.h, store.handle, C.byref(tb), K, mode,
                                             C.byref(opts), C.byref(h)), "agile_session_open")
        return Session(self, h.value, tb.dim)

    # ---- diagnostics
    W_SQ_SLOT, W_SETLOCK, W_WB, W_FILL, W_TICKET, W_WAY, W_CLAIM = 0x01, 0x0A, 0x0B, 0x0D, 0x0E, 0x0F, 0x10

    def debug_lockchain(self, waits: dict, locks: dict, start_wave: int, start_what: int) -> str:
        """Runs the lock-chain walker on a given wait state (agile_debug_lockchain):
        waits = {wave: (kind << 56) | object}, locks = {set: lock word}."""
        n = max(waits) + 1 if waits else 0
        w = np.zeros(n, dtype=np.uint64)
        for k, v in waits.items():
            w[k] = v
        sets = np.array(list(locks.keys()), dtype=np.uint32)
        words = np.array(list(locks.values()), dtype=np.uint32)
        buf = C.create_string_buffer(2048)
        self._check(lib().agile_debug_lockchain(self.h, _ptr(w) if n else 0, n,
                                                _ptr(sets) if sets.size else 0,
                                                _ptr(words) if words.size else 0, sets.size,
                                                start_wave, start_what, buf, 2048),
                    "agile_debug_lockchain")
        return buf.value.decode()

    def debug_trace(self, lines, writes, hit, way, stream=None, store=None):
        store = store or self.store
        self._check(lib().agile_debug_trace(self.h, store.handle, _ptr(lines), _ptr(writes),
                                            lines.numel(), _ptr(hit), _ptr(way), _stream(stream)),
                    "agile_debug_trace")

    COUNTER_NAMES = ("submitted", "completed", "user_done", "work", "requests", "hits",
                     "misses", "reads", "writes", "wb_evict", "wb_flush", "eagain", "sq_spins",
                     "ctrl_cmds", "cq_entries", "aux0", "aux1", "svc_start", "ctrl_fetch",
                     "ctrl_loops", "cq_loops", "wrows", "t_ctrl_fetch", "t_ctrl_copy", "t_ctrl_post",
                     "t_ctrl_hold", "t_ctrl_idle", "ctrl_noroom", "t_cq_busy", "t_cq_idle",
                     "t_u_issue", "t_u_submit", "t_u_wait", "t_u_consume", "tok_lead",
                     "tok_n", "t_u_desc", "t_u_life", "svc_exit", "img_epoch", "work_p1",
                     "work_p2", "work_p3", "work_p4", "work_p5", "work_p6", "work_p7", "defer",
                     "pend", "hit_total", "deflen")

    def debug_counters(self) -> dict:
        n = len(self.COUNTER_NAMES)
        out = (C.c_uint64 * n)()
        lib().agile_debug_counters(self.h, C.cast(out, C.c_void_p), n)
        return dict(zip(self.COUNTER_NAMES, [int(x) for x in out]))

    def debug_dump(self, tags, states, rc, stream=None):
        self._check(lib().agile_debug_dump(self.h, _ptr(tags), _ptr(states), _ptr(rc),
                                           _stream(stream)), "agile_debug_dump")
