"""The operator kernels find the element of a work item (item = element *
nrhs + vector) as trunc((item + 1/2) * fl(1/nrhs)) in FP64 instead of an
integer division; the launch checks items < 2^31 and nrhs <= 64.  This pins
that the truncated FP64 product equals the integer quotient over that whole
range: every nrhs, the items next to every multiple of nrhs near the ends of
the range, and a seeded sample in between (numpy's FP64 arithmetic is the
same IEEE binary64 the kernels use: one rounded addition, one rounded
product)."""
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
