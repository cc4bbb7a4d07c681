"""Pins of the oracle's interleaving over several devices (Sec. 4.3: request i goes to
device i mod n) and of its unit writes (Sec. 3.5's write through the cache, as the
store sees it once done), plus the test helper that lays out device images for the GPU
tests: it must agree with the oracle's layout."""
import numpy as np

import oracle
from gpu_helpers import striped_arrays


def test_three_devices_hand_worked():
    # six one-byte units 10..15 over 3 devices: device d holds units d, d+3
    logical = np.arange(10, 16, dtype=np.uint8)
    d0, d1, d2 = oracle.stripe_split(logical, 3, 1)
    assert d0.tolist() == [10, 13] and d1.tolist() == [11, 14] and d2.tolist() == [12, 15]


def test_two_devices_multi_byte_units_hand_worked():
    # four 2-byte units [0,1] [2,3] [4,5] [6,7] over 2 devices
    logical = np.arange(8, dtype=np.uint8)
    d0, d1 = oracle.stripe_split(logical, 2, 2)
    assert d0.tolist() == [0, 1, 4, 5] and d1.tolist() == [2, 3, 6, 7]


def test_one_device_is_identity_and_every_unit_lands_once():
    rng = np.random.default_rng(1)
    x = rng.integers(0, 256, 64 * 24, dtype=np.uint8)
    (d,) = oracle.stripe_split(x, 1, 64)
    assert np.array_equal(d, x)
    for n in (2, 3, 4, 6):
        devs = oracle.stripe_split(x, n, 64)
        units = {bytes(x[u * 64:(u + 1) * 64]): u for u in range(24)}
        seen = []
        for d, dev in enumerate(devs):
            for k in range(dev.size // 64):
                u = units[bytes(dev[k * 64:(k + 1) * 64])]
                assert u % n == d and u // n == k
                seen.append(u)
        assert sorted(seen) == list(range(24))


def test_helper_layout_equals_oracle():
    rng = np.random.default_rng(2)
    x = rng.integers(0, 256, 4096 * 36, dtype=np.uint8)
    for n in (1, 2, 3, 4):
        ref = oracle.stripe_split(x, n, 4096)
        got = striped_arrays(x, n, 4096)
        assert all(np.array_equal(a, b) for a, b in zip(got, ref))


def test_unit_writes_hand_worked_order():
    img = np.zeros(4 * 2, dtype=np.uint8)
    src = np.array([1, 1, 2, 2, 3, 3], dtype=np.uint8)
    out = oracle.write_units(img, 2, [2, 0, 2], src)
    # unit 2 written twice: the later write (3,3) stays; unit 1 and 3 untouched
    assert out.tolist() == [2, 2, 0, 0, 3, 3, 0, 0]
    assert img.tolist() == [0] * 8  # input not modified
