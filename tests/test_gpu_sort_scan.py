"""GPU checks of the library's own device-wide exclusive scan (BFS edge offsets) and
stable radix sort (the backward pass's occurrence order) against numpy: exact, at sizes
that span one tile (4096 elements), several tiles with a ragged tail, and the recursive
scan of tile sums.  The expected values are numpy's cumulative sum and stable argsort."""
import numpy as np
import pytest

from paper_2504_19365_amd import agile

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [1, 63, 4095, 4096, 4097, 100_003, 20_000_001])
def test_exclusive_scan_u64(n):
    import torch
    rng = np.random.default_rng(n)
    x = rng.integers(0, 1 << 40, size=n, dtype=np.uint64) if n < 10_000_000 else \
        rng.integers(0, 80, size=n, dtype=np.uint64)
    d = torch.from_numpy(x.view(np.int64)).cuda()
    out = torch.empty_like(d)
    agile.exclusive_scan_u64(d, out, n)
    exp = np.zeros(n, dtype=np.uint64)
    np.cumsum(x[:-1], out=exp[1:])
    assert np.array_equal(out.cpu().numpy().view(np.uint64), exp)
    # in place
    agile.exclusive_scan_u64(d, d, n)
    assert np.array_equal(d.cpu().numpy().view(np.uint64), exp)


@pytest.mark.parametrize("n,rowbits", [(1, 3), (64, 1), (4095, 9), (4097, 12), (335_872, 25),
                                       (1_000_003, 17)])
def test_radix_sort_stable_by_row_bits(n, rowbits):
    import torch
    rng = np.random.default_rng(rowbits * 7 + n)
    # the backward pass's keys: (row << 32 | position), positions ascending; Zipf-like rows
    rows = (rng.zipf(1.3, size=n).astype(np.uint64) - 1) % np.uint64(1 << rowbits)
    keys = (rows << np.uint64(32)) | np.arange(n, dtype=np.uint64)
    d = torch.from_numpy(keys.view(np.int64)).cuda()
    agile.radix_sort_u64(d, n, 32, 32 + rowbits)
    order = np.argsort(rows, kind="stable")
    assert np.array_equal(d.cpu().numpy().view(np.uint64), keys[order])


def test_radix_sort_other_bits_ride_along():
    import torch
    rng = np.random.default_rng(1)
    n = 50_000
    keys = rng.integers(0, 1 << 63, size=n, dtype=np.uint64)
    d = torch.from_numpy(keys.view(np.int64)).cuda()
    agile.radix_sort_u64(d, n, 8, 27)
    k = (keys >> np.uint64(8)) & np.uint64((1 << 19) - 1)
    assert np.array_equal(d.cpu().numpy().view(np.uint64), keys[np.argsort(k, kind="stable")])
