"""CPU checks of arithmetic arguments the kernels rely on.

The TSDF kernels take the sensor-frame distances (and the horizontal distance that feeds
the row predicates) as sqrt rounded to nearest, computed from the hardware root, which is
within one ulp, and a correction by its neighbours' residuals (device.h, sqrt_rn).  The
rule is invariant under scaling the argument by 4 while the residuals stay normal, so one
period, every float in [1, 4), with the hardware root off by -1, 0 or +1 ulp, covers it."""
import numpy as np


def _corrected(x, s):
    sm = (s.view(np.uint32) - np.uint32(1)).view(np.float32)
    sp = (s.view(np.uint32) + np.uint32(1)).view(np.float32)
    X = x.astype(np.float64)
    # x - s' s: the product of two floats is exact in fp64, so the difference's sign is exact
    rm = X - sm.astype(np.float64) * s.astype(np.float64)
    rp = X - sp.astype(np.float64) * s.astype(np.float64)
    r = np.where(rm <= 0, sm, s)
    return np.where(rp > 0, sp, r)


def test_sqrt_correction_rule_exhaustive_over_one_period():
    lo, hi = np.float32(1.0).view(np.uint32), np.float32(4.0).view(np.uint32)
    x = np.arange(lo, hi, dtype=np.uint32).view(np.float32)
    want = np.sqrt(x)  # IEEE square root, rounded to nearest
    for off in (-1, 0, 1):
        s = (want.view(np.uint32).astype(np.int64) + off).astype(np.uint32).view(np.float32)
        got = _corrected(x, s)
        assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), off


def test_sqrt_correction_rule_at_range_ends():
    # the kernels take the fast path on [2^-64, FLT_MAX]; its ends and a few scaled values
    x = np.array([2.0 ** -64, 2.0 ** -63 * 3, 1.0, 2.0, 3.0, 2.0 ** 100, 3.4028234e38],
                 dtype=np.float32)
    want = np.sqrt(x)
    for off in (-1, 0, 1):
        s = (want.view(np.uint32).astype(np.int64) + off).astype(np.uint32).view(np.float32)
        assert np.array_equal(_corrected(x, s).view(np.uint32), want.view(np.uint32)), off
