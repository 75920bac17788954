"""The sweep's row set-up takes floor(a / c) for a 32-bit signed a and a cell
count c > 0 as floor((a + 1/2) * fl(1/c)) in FP64 (two roundings, no fused
multiply-add).  The argument: the computed product is within a relative
2^-52 of (a + 1/2) / c, so within |a + 1/2| 2^-52 / c < 1 / (2c) of it, and
(a + 1/2) / c lies at least 1 / (2c) from every integer.  Checked here with
IEEE doubles (Python floats round like the device code) on the values where
a slip would show: multiples of c and their neighbours, the int32 extremes,
and c up to 2^31 - 1."""
import math

import numpy as np


def floor_f(a, c):
    return math.floor((float(a) + 0.5) * (1.0 / float(c)))


def test_floor_division_by_reciprocal_is_exact():
    rng = np.random.default_rng(20241203)
    cs = [1, 2, 3, 5, 7, 42, 105, 1000, 65535, 65536, 1 << 20, (1 << 24) + 1, (1 << 30) + 3, 2 ** 31 - 1]
    cs += [int(c) for c in rng.integers(1, 2 ** 31 - 1, size=40)]
    amin, amax = -(2 ** 31), 2 ** 31 - 1
    n = 0
    for c in cs:
        a_vals = {amin, amin + 1, amax, amax - 1, -1, 0, 1}
        for k in list(range(-4, 5)) + [int(k) for k in rng.integers(amin // c, amax // c + 1, size=20)]:
            for d in (-1, 0, 1):
                a = k * c + d
                if amin <= a <= amax:
                    a_vals.add(a)
        a_vals.update(int(a) for a in rng.integers(amin, amax, size=200, endpoint=True))
        for a in a_vals:
            assert floor_f(a, c) == a // c, (a, c)
            n += 1
    assert n > 10000
