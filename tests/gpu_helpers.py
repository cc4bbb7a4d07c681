"""Shared set-up for the GPU tests: seeded store images in pinned memory and contexts.
Inputs come from the generator module; expected values from the oracle only."""
from __future__ import annotations

import numpy as np

from paper_2504_19365_amd import agile, gen


def device_ready():
    import torch
    return torch.cuda.is_available()


def table_store(rows: int, dim: int, seeds, extra_bytes: int = 0):
    """Pinned image holding len(seeds) concatenated tables (C2 values)."""
    T = len(seeds)
    table_bytes = rows * dim * 4
    nbytes = T * table_bytes + extra_bytes
    nbytes = (nbytes + 4095) // 4096 * 4096
    buf = agile.PinnedBuffer(nbytes)
    for t, s in enumerate(seeds):
        gen.fill_table(buf.ptr + t * table_bytes, 0, rows, dim, s)
    if nbytes > T * table_bytes:
        buf.array[T * table_bytes:] = 0
    return buf


def striped_arrays(logical, n: int, unit_bytes: int):
    """Device images of a logical image laid out unit by unit over n devices (unit u of
    the logical image is unit u // n of device u % n), as host arrays."""
    x = np.ascontiguousarray(logical).view(np.uint8).reshape(-1, n, unit_bytes)
    return [np.ascontiguousarray(x[:, d, :]).ravel() for d in range(n)]


def striped_store(logical, n: int, unit_bytes: int):
    """Pinned device images (one PinnedBuffer each) of a logical image."""
    bufs = []
    for a in striped_arrays(logical, n, unit_bytes):
        b = agile.PinnedBuffer(a.size)
        b.array[:] = a
        bufs.append(b)
    return bufs


def cuda(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


class DeviceArray:
    """__cuda_array_interface__ view of device memory owned by the library."""

    def __init__(self, ptr: int, nbytes: int):
        self.__cuda_array_interface__ = {"shape": (nbytes,), "typestr": "|u1",
                                         "data": (ptr, False), "version": 3, "strides": None}


def device_bytes(ptr: int, nbytes: int):
    import torch
    return torch.as_tensor(DeviceArray(ptr, nbytes), device="cuda")


def dump_meta(ctx):
    import torch
    n = ctx.info()["num_lines"]
    tags = torch.empty(n, dtype=torch.int64, device="cuda")
    st = torch.empty(n, dtype=torch.uint8, device="cuda")
    rc = torch.empty(n, dtype=torch.int32, device="cuda")
    ctx.debug_dump(tags, st, rc)
    return tags.cpu().numpy(), st.cpu().numpy(), rc.cpu().numpy()


def check_quiescent_invariants(ctx, assoc: int):
    """No line id resident in two ways; no pins; nothing in flight (Sec. 3.4)."""
    tags, st, rc = dump_meta(ctx)
    valid = tags[tags >= 0]
    assert valid.size == np.unique(valid).size, "a line id is resident in two ways"
    assert np.all(rc == 0), "pins left at quiescence"
    assert np.all((st == 0) | (st == 2) | (st == 3)), "lines still in flight at quiescence"
    sets = tags.size // assoc
    idx = np.nonzero(tags >= 0)[0]
    assert np.all(tags[idx] % sets == idx // assoc), "a line sits in the wrong set"
    return tags, st
