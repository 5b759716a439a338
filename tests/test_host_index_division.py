"""The integer identity behind the batched FFT passes' index division (no GPU needed).

For a divisor d that is not a power of two and m = floor((2^32 - 1) / d) + 1, the high 32 bits of
x m equal floor(x / d) whenever x d < 2^32.  The batched passes divide element, butterfly and
sequence indices this way; these checks cover every dividend below 4096 for every divisor up to
4096 (the element and butterfly ranges), random pairs up to the bound, and show that the bound is
needed (the identity fails beyond it for some pairs)."""
import numpy as np


def magic(d):
    return (0xFFFFFFFF // d + 1) & 0xFFFFFFFF


def mulhi_div(x, d):
    return (x.astype(np.uint64) * np.uint64(magic(d))) >> np.uint64(32)


def test_small_ranges_exhaustive():
    x = np.arange(4096, dtype=np.uint64)
    for d in range(3, 4097):
        if d & (d - 1) == 0:
            continue
        np.testing.assert_array_equal(mulhi_div(x, d), x // np.uint64(d), err_msg=f"d={d}")


def test_random_pairs_within_bound():
    rng = np.random.default_rng(7)
    for _ in range(2000):
        d = int(rng.integers(3, 1 << 20))
        if d & (d - 1) == 0:
            continue
        xmax = ((1 << 32) - 1) // d          # x d < 2^32
        x = rng.integers(0, xmax + 1, size=512, dtype=np.uint64)
        x[:2] = [xmax, max(xmax - 1, 0)]
        np.testing.assert_array_equal(mulhi_div(x, d), x // np.uint64(d), err_msg=f"d={d}")


def test_bound_is_needed():
    # beyond x d < 2^32 the product can round up past the next multiple of d
    rng = np.random.default_rng(11)
    failures = 0
    for _ in range(200):
        d = int(rng.integers(1 << 12, 1 << 16)) | 1
        x = rng.integers(1 << 28, 1 << 32, size=4096, dtype=np.uint64)
        failures += int(np.count_nonzero(mulhi_div(x, d) != x // np.uint64(d)))
    assert failures > 0
