"""The division-free quotient of the march (csrc/march.h small_quot), emulated
in FP32 on the CPU: q = trunc((n + 1/2) * r) with r the reciprocal of d to
within one ulp either side (the hardware rcp is within 1 ulp).  It must equal
n // d wherever the kernels use it: brick and super-brick indices of a chunk
(n < 64, d <= 64) and the staging columns of an LDS box (n < 2^14,
d < 2^10), all inside the stated n + d < 2^20."""
import numpy as np


def _quot(n, d, ulp):
    r = (np.float32(1.0) / d.astype(np.float32))
    if ulp:
        r = np.nextafter(r, np.float32(np.inf) if ulp > 0 else np.float32(0.0)).astype(np.float32)
    v = (n.astype(np.float32) + np.float32(0.5)) * r
    return np.trunc(v.astype(np.float32)).astype(np.int64)


def _check(n_max, d_max):
    n = np.arange(n_max, dtype=np.int64)
    for d0 in range(1, d_max + 1):
        d = np.full_like(n, d0)
        want = n // d0
        for ulp in (-1, 0, 1):
            assert np.array_equal(_quot(n, d, ulp), want), (d0, ulp)


def test_chunk_brick_indices():
    _check(64, 64)


def test_staging_columns():
    # every divisor up to 1023 for all n < 2^14
    _check(1 << 14, 1023)


def test_bound_is_where_it_fails_first():
    # near n + d = 2^24 the margin is gone: the check is not vacuous
    n = np.arange((1 << 24) - 4096, 1 << 24, dtype=np.int64)
    bad = 0
    for d0 in (3, 7, 11, 13):
        d = np.full_like(n, d0)
        for ulp in (-1, 1):
            bad += int((_quot(n, d, ulp) != n // d0).sum())
    assert bad > 0
