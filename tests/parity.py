"""Comparison helpers for the parity tests.

Both sides compare single-precision distances (section 6.1).  The oracle takes
the exact distance (fp64) and rounds it once to fp32; the library computes the
same correctly rounded value with compensated fp32 arithmetic on the device and
fp64 accumulation on the host.  The two can differ only when the exact value
lies within the accumulation error (about 2^-44 relative on the device,
D * 2^-53 on the host) of a midpoint between two floats, and then by one unit
in the last place.  So:

* distances: at most 1 ulp apart, and identical on all but a tiny fraction;
* ids: identical, except where a decision of the search was decided by a gap
  of at most two ulps (the oracle's near-tie margin) and a one-ulp difference
  can flip it.
"""

import numpy as np

ULP = 2.0 ** -23  # relative size of one fp32 ulp, upper bound
TIE = 2 * ULP     # near-tie margin below which an id divergence is allowed
MAX_NONIDENTICAL = 1e-4  # largest fraction of distances allowed to differ (by 1 ulp)


def _ordered(a):
    """float32 values as integers with the same order (sign-magnitude -> two's complement)."""
    i = np.ascontiguousarray(np.asarray(a, dtype=np.float32)).view(np.int32).astype(np.int64)
    return np.where(i < 0, -(i & 0x7FFFFFFF), i)


def ulp_diff(a, b):
    """|a - b| in fp32 units in the last place (inf == inf counts as 0)."""
    a = np.asarray(a, dtype=np.float32)
    b = np.asarray(b, dtype=np.float32)
    same = (a == b) | (np.isinf(a) & np.isinf(b) & (np.sign(a) == np.sign(b)))
    return np.where(same, 0, np.abs(_ordered(a) - _ordered(b)))


class DistTally:
    """Counts compared and non-identical distances; every pair must be within 1 ulp."""

    def __init__(self):
        self.n = 0
        self.off = 0

    def check(self, got, want, what=""):
        u = ulp_diff(got, want)
        assert (u <= 1).all(), (what, np.asarray(got)[u > 1][:4], np.asarray(want)[u > 1][:4])
        self.n += u.size
        self.off += int((u != 0).sum())

    def done(self):
        assert self.off <= max(1, MAX_NONIDENTICAL * self.n), (self.off, self.n)
        return self.off
