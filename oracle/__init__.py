"""CPU oracle for the asynchronous block-I/O path (ctypes wrapper over liboracle.so).

TEST INFRASTRUCTURE: only tests/, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path never routes through it.  See
oracle.h for the definitions each function follows and the pins that check them.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain C, single-threaded, no fused multiply-adds
    other than explicit fmaf)."""
    if force or not os.path.exists(LIB_PATH):
        # oracle.c has no OpenMP pragma: -fopenmp only builds the all-cores baseline loop
        # of cpu_baseline.c
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-fopenmp", "-shared", "-o", LIB_PATH + ".tmp", os.path.join(_HERE, "oracle.c"),
               os.path.join(_HERE, "cpu_baseline.c"), "-lm"]
        subprocess.check_call(cmd)
        os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=False)
        L = C.CDLL(LIB_PATH)
        u64, u32, i64, vp, dbl, f32 = (C.c_uint64, C.c_uint32, C.c_int64, C.c_void_p,
                                       C.c_double, C.c_float)
        L.oracle_fK.restype = f32
        L.oracle_fK.argtypes = [f32, u32]
        L.oracle_gather.argtypes = [vp, u64, vp, u64, vp]
        L.oracle_embbag_forward.argtypes = [vp, u64, u32, u32, vp, vp, u64, u32, vp, u64, vp]
        L.oracle_embbag_forward_par.argtypes = [vp, u64, u32, u32, vp, vp, u64, u32, vp]
        L.oracle_par_threads.restype = C.c_int
        L.oracle_embbag_backward_sgd.restype = u64
        L.oracle_embbag_backward_sgd.argtypes = [vp, u64, u32, u32, vp, vp, u64, vp, f32]
        L.oracle_bfs.argtypes = [vp, vp, u64, i64, vp]
        L.oracle_bfs_validate.restype = C.c_int
        L.oracle_bfs_validate.argtypes = [vp, vp, u64, i64, vp]
        L.oracle_spmv.argtypes = [vp, vp, vp, vp, u64, u64, vp]
        L.oracle_clock_new.restype = vp
        L.oracle_clock_new.argtypes = [u32, u32]
        L.oracle_clock_free.argtypes = [vp]
        L.oracle_clock_access.restype = C.c_int
        L.oracle_clock_access.argtypes = [vp, u64, C.c_int, C.POINTER(C.c_int32)]
        L.oracle_clock_run.argtypes = [vp, vp, vp, u64, vp, vp]
        L.oracle_stripe_split.argtypes = [vp, u64, u64, u32, vp]
        L.oracle_write_units.argtypes = [vp, u64, vp, u64, vp]
        L.oracle_clock_flush.restype = u64
        L.oracle_clock_flush.argtypes = [vp]
        L.oracle_clock_counters.argtypes = [vp, vp]
        L.oracle_clock_state.argtypes = [vp, vp, vp]
        L.oracle_eq1.restype = dbl
        L.oracle_eq1.argtypes = [dbl]
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return C.c_void_p(0)
    if isinstance(a, np.ndarray):
        assert a.flags.c_contiguous
        return C.c_void_p(a.ctypes.data)
    return C.c_void_p(int(a))


def fK(v: float, K: int) -> float:
    return float(lib().oracle_fK(C.c_float(v), K))


def gather(image: np.ndarray, row_bytes: int, rows: np.ndarray) -> np.ndarray:
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.empty((rows.size, row_bytes), dtype=np.uint8)
    lib().oracle_gather(_p(image), row_bytes, _p(rows), rows.size, _p(out))
    return out


def embbag_forward_par(image, rows: int, dim: int, T: int, idx, off, B: int, K: int) -> np.ndarray:
    """All bags, spread over the cores (the all-cores CPU baseline)."""
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    off = np.ascontiguousarray(off, dtype=np.int64)
    out = np.empty((B * T, dim), dtype=np.float32)
    lib().oracle_embbag_forward_par(_p(image), rows, dim, T, _p(idx), _p(off), B, K, _p(out))
    return out


def par_threads() -> int:
    return int(lib().oracle_par_threads())


def embbag_forward(image, rows: int, dim: int, T: int, idx, off, B: int, K: int,
                   bags=None) -> np.ndarray:
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    off = np.ascontiguousarray(off, dtype=np.int64)
    if bags is not None:
        bags = np.ascontiguousarray(bags, dtype=np.int64)
        n = bags.size
    else:
        n = B * T
    out = np.empty((n, dim), dtype=np.float32)
    lib().oracle_embbag_forward(_p(image), rows, dim, T, _p(idx), _p(off), B, K, _p(bags),
                                0 if bags is None else bags.size, _p(out))
    return out


def embbag_backward_sgd(image: np.ndarray, rows: int, dim: int, T: int, idx, off, B: int,
                        grad_out: np.ndarray, lr: float) -> int:
    """Updates `image` in place; returns the number of distinct rows touched."""
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    off = np.ascontiguousarray(off, dtype=np.int64)
    g = np.ascontiguousarray(grad_out, dtype=np.float32)
    return int(lib().oracle_embbag_backward_sgd(_p(image), rows, dim, T, _p(idx), _p(off), B,
                                                _p(g), C.c_float(lr)))


def bfs(row_ptr, col, src: int) -> np.ndarray:
    V = row_ptr.size - 1
    level = np.empty(V, dtype=np.int32)
    lib().oracle_bfs(_p(row_ptr), _p(col), V, src, _p(level))
    return level


def bfs_validate(row_ptr, col, src: int, level) -> int:
    return int(lib().oracle_bfs_validate(_p(row_ptr), _p(col), row_ptr.size - 1, src,
                                         _p(np.ascontiguousarray(level, dtype=np.int32))))


def spmv(row_ptr, col, val, x, r0: int = 0, r1=None) -> np.ndarray:
    if r1 is None:
        r1 = row_ptr.size - 1
    y = np.empty(max(r1 - r0, 0), dtype=np.float32)
    lib().oracle_spmv(_p(row_ptr), _p(col), _p(val), _p(x), r0, r1, _p(y))
    return y


class Clock:
    """Sequential clock (second-chance) cache simulator."""

    def __init__(self, sets: int, assoc: int):
        self.sets, self.assoc = sets, assoc
        self._h = lib().oracle_clock_new(sets, assoc)

    def __del__(self):
        if getattr(self, "_h", None):
            lib().oracle_clock_free(self._h)
            self._h = None

    def access(self, line: int, write: bool = False):
        w = C.c_int32(-1)
        hit = lib().oracle_clock_access(self._h, line, 1 if write else 0, C.byref(w))
        return bool(hit), int(w.value)

    def run(self, lines, writes=None):
        lines = np.ascontiguousarray(lines, dtype=np.uint64)
        hit = np.empty(lines.size, dtype=np.uint8)
        way = np.empty(lines.size, dtype=np.int32)
        wr = None if writes is None else np.ascontiguousarray(writes, dtype=np.uint8)
        lib().oracle_clock_run(self._h, _p(lines), _p(wr), lines.size, _p(hit), _p(way))
        return hit, way

    def flush(self) -> int:
        return int(lib().oracle_clock_flush(self._h))

    def counters(self) -> dict:
        c = np.zeros(4, dtype=np.uint64)
        lib().oracle_clock_counters(self._h, _p(c))
        return dict(hits=int(c[0]), misses=int(c[1]), wb_evict=int(c[2]), wb_flush=int(c[3]))

    def state(self):
        n = self.sets * self.assoc
        tags = np.empty(n, dtype=np.int64)
        dirty = np.empty(n, dtype=np.uint8)
        lib().oracle_clock_state(self._h, _p(tags), _p(dirty))
        return tags.reshape(self.sets, self.assoc), dirty.reshape(self.sets, self.assoc)


def eq1(ctc: float) -> float:
    return float(lib().oracle_eq1(ctc))


def stripe_split(logical: np.ndarray, n: int, unit_bytes: int) -> list:
    """Device images of a logical image interleaved unit by unit over n devices."""
    logical = np.ascontiguousarray(logical).view(np.uint8).ravel()
    units = logical.size // unit_bytes
    assert units * unit_bytes == logical.size and units % n == 0
    devs = [np.empty(units // n * unit_bytes, dtype=np.uint8) for _ in range(n)]
    ptrs = (C.c_void_p * n)(*[d.ctypes.data for d in devs])
    lib().oracle_stripe_split(_p(logical), units, unit_bytes, n, ptrs)
    return devs


def write_units(image: np.ndarray, unit_bytes: int, lines, src) -> np.ndarray:
    """A copy of image after writing src[i] to unit lines[i], in order."""
    out = np.array(np.ascontiguousarray(image).view(np.uint8).ravel())
    lines = np.ascontiguousarray(lines, dtype=np.uint64)
    src = np.ascontiguousarray(src).view(np.uint8).ravel()
    assert src.size == lines.size * unit_bytes and (lines.size == 0 or int(lines.max()) < out.size // unit_bytes)
    lib().oracle_write_units(_p(out), unit_bytes, _p(lines), lines.size, _p(src))
    return out
