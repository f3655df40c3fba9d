"""The operator kernels divide by run-time sizes in FP64 instead of integer
division: the element of a work item (item = element * nrhs + vector) is
trunc((item + 1/2) * fl(1/nrhs)), and an element's coordinates come from
the same form with 1/Nx and 1/Ny; the launch checks items < 2^31 and
nrhs <= 64, the level element counts < 2^31.  This pins that the truncated
FP64 product equals the integer quotient over those ranges: every nrhs, the
items next to multiples of the divisor near the ends of the range, and
seeded samples in between (numpy's FP64 arithmetic is the same IEEE
binary64 the kernels use: one rounded addition, one rounded product)."""
import numpy as np


def fp64_quotient(item, d):
    return np.trunc((item.astype(np.float64) + 0.5) * (1.0 / d)).astype(np.int64)


def test_fp64_item_quotient_is_exact():
    rng = np.random.default_rng(20191004)
    top = (1 << 31) - 1
    for d in range(2, 65):
        q_hi = top // d
        mult = np.concatenate([np.arange(0, 4096), np.arange(q_hi - 4096, q_hi + 1),
                               rng.integers(0, q_hi + 1, 20000)]) * d
        item = np.concatenate([mult - 1, mult, mult + 1, mult + d - 1])
        item = item[(item >= 0) & (item <= top)]
        assert np.array_equal(fp64_quotient(item, d), item // d), d


def test_fp64_quotient_by_mesh_sizes_is_exact():
    """The same form divides element indices (< 2^31) by the mesh's Nx and
    Ny: every divisor 1..4096 and a seeded sample of larger ones up to 2^31,
    at the items next to multiples of the divisor."""
    rng = np.random.default_rng(20191005)
    top = (1 << 31) - 1
    divisors = np.concatenate([np.arange(1, 4097), rng.integers(4097, top, 2000)])
    for d in divisors:
        d = int(d)
        q_hi = top // d
        q = np.concatenate([np.arange(0, min(q_hi, 64) + 1), rng.integers(0, q_hi + 1, 64),
                            np.arange(max(q_hi - 64, 0), q_hi + 1)])
        item = np.concatenate([q * d - 1, q * d, q * d + 1, q * d + d - 1])
        item = item[(item >= 0) & (item <= top)]
        assert np.array_equal(fp64_quotient(item, d), item // d), d
