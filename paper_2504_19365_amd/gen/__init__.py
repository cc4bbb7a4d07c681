"""Seeded synthetic input generators (ctypes wrapper over libagilegen.so).

Only inputs are produced here: table contents, lookup indices, bag lengths, RMAT CSR
graphs, dense vectors, gradients and request streams.  Both the GPU path and the CPU
oracle consume these; nothing of the method's arithmetic lives in this module.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libagilegen.so")

S_VALUES, S_ZIPF, S_BAGLEN, S_RMAT, S_RELABEL, S_X, S_GRAD, S_ARRIVAL, S_REQSIZE, S_SRC, \
    S_BLOCKS, S_VAL = range(1, 13)

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        u64, u32, i64, dbl, vp = C.c_uint64, C.c_uint32, C.c_int64, C.c_double, C.c_void_p
        L.gen_u64.restype = u64
        L.gen_u64.argtypes = [u64, u32, u64]
        L.gen_u01.restype = dbl
        L.gen_u01.argtypes = [u64, u32, u64]
        L.gen_fill_table.argtypes = [vp, u64, u64, u32, u64]
        L.gen_zipf_cum.argtypes = [vp, u64, dbl]
        L.gen_zipf_pick.restype = i64
        L.gen_zipf_pick.argtypes = [vp, u64, dbl]
        L.gen_zipf_rows.argtypes = [vp, u64, u64, u64, u64, vp]
        L.gen_uniform_int.argtypes = [u64, u32, u64, u64, i64, i64, vp]
        L.gen_embbag_batch.restype = u64
        L.gen_embbag_batch.argtypes = [vp, u64, u64, u32, u32, u32, u64, vp, vp]
        L.gen_uniform_f32.argtypes = [u64, u32, u64, dbl, dbl, vp]
        L.gen_normal_f32.argtypes = [u64, u64, vp]
        L.gen_rmat_degrees.argtypes = [u32, u32, dbl, dbl, dbl, u64, vp]
        L.gen_rmat_fill.argtypes = [u32, u32, dbl, dbl, dbl, u64, vp, vp, vp]
        L.gen_bfs_source.restype = i64
        L.gen_bfs_source.argtypes = [u64, vp, u64]
        L.gen_uniform_blocks.argtypes = [u64, u64, u64, vp]
        L.gen_requests.argtypes = [u64, u64, dbl, u32, vp, vp]
        L.gen_num_threads.restype = C.c_int
        _lib = L
    return _lib


def _p(a):
    return C.c_void_p(a.ctypes.data) if isinstance(a, np.ndarray) else C.c_void_p(int(a))


def u64(seed: int, stream: int, i: int) -> int:
    return int(lib().gen_u64(seed, stream, i))


def u01(seed: int, stream: int, i: int) -> float:
    return float(lib().gen_u01(seed, stream, i))


def fill_table(dst_ptr: int, row0: int, nrows: int, dim: int, seed: int) -> None:
    """Write rows [row0, row0+nrows) of table `seed` (dim columns, fp32) at dst_ptr."""
    lib().gen_fill_table(_p(dst_ptr), row0, nrows, dim, seed)


def table(rows: int, dim: int, seed: int) -> np.ndarray:
    out = np.empty((rows, dim), dtype=np.float32)
    lib().gen_fill_table(_p(out), 0, rows, dim, seed)
    return out


def zipf_cum(n: int, alpha: float) -> np.ndarray:
    cum = np.empty(n, dtype=np.float64)
    lib().gen_zipf_cum(_p(cum), n, alpha)
    return cum


def zipf_pick(cum: np.ndarray, u: float) -> int:
    return int(lib().gen_zipf_pick(_p(cum), cum.size, u))


def zipf_rows(cum: np.ndarray, seed: int, count: int, i0: int = 0) -> np.ndarray:
    out = np.empty(count, dtype=np.int64)
    lib().gen_zipf_rows(_p(cum), cum.size, seed, i0, count, _p(out))
    return out


def uniform_int(seed: int, stream: int, count: int, lo: int, hi: int, i0: int = 0) -> np.ndarray:
    out = np.empty(count, dtype=np.int64)
    lib().gen_uniform_int(seed, stream, i0, count, lo, hi, _p(out))
    return out


def embbag_batch(cum: np.ndarray, B: int, T: int, len_lo: int, len_hi: int, seed: int):
    """Returns (offsets int64[B*T+1], idx int64[n]) in sample-major bag order."""
    offsets = np.empty(B * T + 1, dtype=np.int64)
    n = int(lib().gen_embbag_batch(_p(cum), cum.size, B, T, len_lo, len_hi, seed, _p(offsets),
                                   C.c_void_p(0)))
    idx = np.empty(max(n, 1), dtype=np.int64)
    lib().gen_embbag_batch(_p(cum), cum.size, B, T, len_lo, len_hi, seed, _p(offsets), _p(idx))
    return offsets, idx[:n]


def uniform_f32(seed: int, stream: int, count: int, lo: float, hi: float) -> np.ndarray:
    out = np.empty(count, dtype=np.float32)
    lib().gen_uniform_f32(seed, stream, count, lo, hi, _p(out))
    return out


def normal_f32(seed: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.float32)
    lib().gen_normal_f32(seed, count, _p(out))
    return out


def rmat_degrees(scale: int, edge_factor: int, a: float, b: float, c: float, seed: int):
    deg = np.empty(1 << scale, dtype=np.uint32)
    lib().gen_rmat_degrees(scale, edge_factor, a, b, c, seed, _p(deg))
    return deg


def rmat_fill(scale, edge_factor, a, b, c, seed, row_ptr_ptr, col_ptr, val_ptr):
    """Pass 2 into caller-provided memory (pointers or numpy arrays)."""
    lib().gen_rmat_fill(scale, edge_factor, a, b, c, seed, _p(row_ptr_ptr), _p(col_ptr),
                        _p(val_ptr) if val_ptr is not None else C.c_void_p(0))


def rmat_csr(scale: int, edge_factor: int, a: float, b: float, c: float, seed: int):
    """Small graphs only: returns numpy (row_ptr int64, col int32, val fp32)."""
    deg = rmat_degrees(scale, edge_factor, a, b, c, seed)
    row_ptr = np.zeros((1 << scale) + 1, dtype=np.int64)
    np.cumsum(deg, out=row_ptr[1:])
    E = int(row_ptr[-1])
    col = np.empty(max(E, 1), dtype=np.int32)
    val = np.empty(max(E, 1), dtype=np.float32)
    rmat_fill(scale, edge_factor, a, b, c, seed, row_ptr, col, val)
    return row_ptr, col[:E], val[:E]


def bfs_source(seed: int, row_ptr: np.ndarray) -> int:
    return int(lib().gen_bfs_source(seed, _p(row_ptr), row_ptr.size - 1))


def uniform_blocks(seed: int, count: int, nblocks: int) -> np.ndarray:
    out = np.empty(count, dtype=np.int64)
    lib().gen_uniform_blocks(seed, count, nblocks, _p(out))
    return out


def requests(seed: int, count: int, rate: float, max_log2: int = 12):
    t = np.empty(count, dtype=np.float64)
    n = np.empty(count, dtype=np.int64)
    lib().gen_requests(seed, count, rate, max_log2, _p(t), _p(n))
    return t, n


def num_threads() -> int:
    return int(lib().gen_num_threads())


def rmat_layout(scale: int, edge_factor: int, a: float, b: float, c: float, seed: int):
    """Pass 1 of the RMAT generator and the store layout of the CSR arrays:
    [row_ptr int64 (V+1)] [pad to 4 KiB] [col int32 E] [pad] [val fp32 E] [pad].
    Returns (row_ptr numpy int64, dict of byte offsets and total size)."""
    deg = rmat_degrees(scale, edge_factor, a, b, c, seed)
    V = 1 << scale
    row_ptr = np.zeros(V + 1, dtype=np.int64)
    np.cumsum(deg, out=row_ptr[1:])
    del deg
    E = int(row_ptr[-1])
    up = lambda v: (v + 4095) // 4096 * 4096  # noqa: E731
    rp_off = 0
    col_off = up(8 * (V + 1))
    val_off = up(col_off + 4 * E)
    total = up(val_off + 4 * E)
    return row_ptr, dict(V=V, E=E, row_ptr_offset=rp_off, col_offset=col_off, val_offset=val_off,
                         total=total)


def rmat_fill_store(base_ptr: int, row_ptr: np.ndarray, lay: dict, scale: int, edge_factor: int,
                    a: float, b: float, c: float, seed: int) -> None:
    """Pass 2: writes row_ptr, col and val into the store image at base_ptr."""
    import ctypes as _C
    V = lay["V"]
    _C.memmove(base_ptr + lay["row_ptr_offset"], row_ptr.ctypes.data, 8 * (V + 1))
    rmat_fill(scale, edge_factor, a, b, c, seed, base_ptr + lay["row_ptr_offset"],
              base_ptr + lay["col_offset"], base_ptr + lay["val_offset"])


def serve_stream(count: int, rate: float, rows: int, alpha: float, seed: int,
                 max_log2: int = 12, bag_hi: int = 80):
    """Request stream for the serving workload: Poisson arrivals (mean gap 1/rate),
    request sizes n = clamp(round(2^(max_log2 * u)), 1, 2^max_log2), each request split
    into consecutive bags of length uniform [1, bag_hi] (the last one truncated), rows
    Zipf(alpha).  Returns (arrival_s, req_bag0[count+1], bag_off[nbags+1], idx)."""
    arrival, size = requests(seed, count, rate, max_log2)
    total = int(size.sum())
    lens = uniform_int(seed, S_BAGLEN, total, 1, bag_hi)  # more than enough draws
    req_bag0 = np.zeros(count + 1, dtype=np.int64)
    bag_lens = []
    k = 0
    for r in range(count):
        left = int(size[r])
        nb = 0
        while left > 0:
            L = min(int(lens[k]), left)
            k += 1
            bag_lens.append(L)
            left -= L
            nb += 1
        req_bag0[r + 1] = req_bag0[r] + nb
    bag_off = np.zeros(len(bag_lens) + 1, dtype=np.int64)
    np.cumsum(np.asarray(bag_lens, dtype=np.int64), out=bag_off[1:])
    idx = zipf_rows(zipf_cum(rows, alpha), seed, total)
    return arrival, req_bag0, bag_off, idx
