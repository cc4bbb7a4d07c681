"""GPU parity of the out-of-HBM graph workloads: BFS levels (bit-exact) and CSR SpMV
(bit-exact: the same fmaf fold order as the plain definition) with the CSR arrays held in
the emulated store and read through the HBM cache.  Expected values from the oracle."""
import numpy as np
import pytest

import oracle
from paper_2504_19365_amd import agile, gen

from gpu_helpers import check_quiescent_invariants, cuda

pytestmark = pytest.mark.gpu

ABC = (0.57, 0.19, 0.19)


def _graph(scale, ef, seed=0):
    row_ptr, lay = gen.rmat_layout(scale, ef, *ABC, seed)
    buf = agile.PinnedBuffer(lay["total"])
    gen.rmat_fill_store(buf.ptr, row_ptr, lay, scale, ef, *ABC, seed)
    V, E = lay["V"], lay["E"]
    img = buf.array
    col = img[lay["col_offset"]:lay["col_offset"] + 4 * E].view(np.int32)
    val = img[lay["val_offset"]:lay["val_offset"] + 4 * E].view(np.float32)
    g = agile.CSR(V, E, lay["row_ptr_offset"], lay["col_offset"], lay["val_offset"])
    return buf, g, row_ptr, col, val


@pytest.mark.parametrize("scale,ef,cache_kw", [
    (12, 16, dict(cache_bytes=64 << 10, assoc=4)),
    (16, 16, dict(cache_bytes=1 << 20, assoc=8)),
    (20, 16, dict(cache_bytes=64 << 20, assoc=16)),
    # multi-block lines: one command moves 4 or 16 blocks; SpMV windows sized by the sets
    (18, 16, dict(cache_bytes=4 << 20, assoc=4, line_bytes=16384)),
    (20, 16, dict(cache_bytes=64 << 20, assoc=16, line_bytes=65536)),
    # 32 blocks per command (the SpMV line size of the scale-26 measurement), roomy and
    # with 16 lines in 4 sets
    (20, 16, dict(cache_bytes=64 << 20, assoc=16, line_bytes=131072)),
    (18, 16, dict(cache_bytes=2 << 20, assoc=4, line_bytes=131072)),
])
def test_bfs_and_spmv_bit_exact(scale, ef, cache_kw):
    import torch
    buf, g, row_ptr, col, val = _graph(scale, ef)
    kw = dict(line_bytes=4096, num_qp=8, qp_depth=256, timeout_ns=int(10e9))
    kw.update(cache_kw)
    ctx = agile.Context(**kw)
    try:
        ctx.open_store(buf)
        src = gen.bfs_source(0, row_ptr)
        level = torch.empty(g.num_vertices, dtype=torch.int32, device="cuda")
        nl = ctx.bfs(g, src, level)
        got = level.cpu().numpy()
        ref = oracle.bfs(row_ptr, col, src)
        assert np.array_equal(got, ref)
        assert oracle.bfs_validate(row_ptr, col, src, got) == 0
        assert nl == int(ref.max()) + 1
        x = gen.uniform_f32(1, gen.S_X, g.num_vertices, -1.0, 1.0)
        y = torch.empty(g.num_vertices, dtype=torch.float32, device="cuda")
        ctx.spmv(g, cuda(x), y)
        ctx.sync()
        yref = oracle.spmv(row_ptr, col, val, x)
        assert np.array_equal(y.cpu().numpy().view(np.uint32), yref.view(np.uint32))
        check_quiescent_invariants(ctx, cache_kw["assoc"])
    finally:
        ctx.close_store()
        ctx.shutdown()
        buf.free()


def test_bfs_from_isolated_and_leaf_sources():
    import torch
    buf, g, row_ptr, col, val = _graph(10, 4)
    ctx = agile.Context(cache_bytes=1 << 20, line_bytes=4096, assoc=8, num_qp=2, qp_depth=64,
                        timeout_ns=int(5e9))
    try:
        ctx.open_store(buf)
        deg = np.diff(row_ptr)
        for src in [int(np.nonzero(deg == 0)[0][0]), int(np.argmax(deg))]:
            level = torch.empty(g.num_vertices, dtype=torch.int32, device="cuda")
            ctx.bfs(g, src, level)
            assert np.array_equal(level.cpu().numpy(), oracle.bfs(row_ptr, col, src))
    finally:
        ctx.close_store()
        ctx.shutdown()
        buf.free()


@pytest.mark.parametrize("scale", [12, 18])
def test_resident_kernels_equal_oracle_and_cached(scale):
    """The kernel-only baselines (the same BFS and SpMV kernels over a copy of the store
    image resident in HBM, no cache) give the oracle's levels and fold bit for bit, and
    leave the context usable for cached runs afterwards."""
    import torch
    buf, g, row_ptr, col, val = _graph(scale, 16)
    ctx = agile.Context(cache_bytes=1 << 20, line_bytes=4096, assoc=8, num_qp=4, qp_depth=256,
                        timeout_ns=int(10e9))
    try:
        ctx.open_store(buf)
        dimg = torch.from_numpy(buf.array.view(np.uint8)).cuda()
        src = gen.bfs_source(0, row_ptr)
        level = torch.empty(g.num_vertices, dtype=torch.int32, device="cuda")
        nl = ctx.bfs_resident(dimg, buf.nbytes, g, src, level)
        ref = oracle.bfs(row_ptr, col, src)
        assert np.array_equal(level.cpu().numpy(), ref) and nl == int(ref.max()) + 1
        x = gen.uniform_f32(1, gen.S_X, g.num_vertices, -1.0, 1.0)
        y = torch.empty(g.num_vertices, dtype=torch.float32, device="cuda")
        ctx.spmv_resident(dimg, buf.nbytes, g, cuda(x), y)
        ctx.sync()
        exp = oracle.spmv(row_ptr, col, val, x, 0, g.num_vertices)
        assert np.array_equal(y.cpu().numpy().view(np.uint32), exp.view(np.uint32))
        # the cached kernels still run after the resident ones (work counters cleared)
        y2 = torch.empty_like(y)
        ctx.spmv(g, cuda(x), y2)
        ctx.sync()
        assert torch.equal(y, y2)
        check_quiescent_invariants(ctx, 8)
    finally:
        ctx.close_store()
        ctx.shutdown()
        buf.free()
