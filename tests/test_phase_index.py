"""The float64 kernels' phasor-table index, emulated on the CPU.

The float64 bin loops carry the phase tu in units of 1/2048 cycle, take n = rint(tu) by adding
and subtracting 1.5 * 2^52, index the table with the low 11 bits of the sum and rotate the entry
by the remainder y = tu - n. This checks that arithmetic with numpy float64 (the same IEEE
operations) against exact integer arithmetic, at phases well beyond 2^31 table units, where a
float64 -> int32 conversion would clamp, and that the set-up's phase limit keeps tu in range.
"""
import numpy as np

RND = 6755399441055744.0   # 1.5 * 2^52
PH_TBL = 2048
PHASE_LIMIT = 2.0 ** 39    # cycles


def kernel_index(tu):
    tu = np.asarray(tu, dtype=np.float64)
    t = tu + RND
    n = t - RND
    y = tu - n
    idx = t.view(np.int64) & (PH_TBL - 1)     # the low word of t; its low 11 bits
    return idx, n, y


def test_index_and_remainder_are_exact_beyond_int32():
    rng = np.random.default_rng(0)
    tu = np.concatenate([
        rng.uniform(-1e4, 1e4, 2000),
        2.0 ** 31 + rng.uniform(-3e3, 3e3, 2000),
        -(2.0 ** 31) + rng.uniform(-3e3, 3e3, 2000),
        rng.uniform(-(2.0 ** 50), 2.0 ** 50, 2000),
        np.array([0.5, 1.5, 2.5, -0.5, -1.5, 2.0 ** 31 + 0.5, 2047.5, -2048.5]),
    ])
    idx, n, y = kernel_index(tu)
    want_n = np.rint(tu)                                 # ties to even, as the addition rounds
    np.testing.assert_array_equal(n, want_n)
    exact_mod = np.array([int(v) % PH_TBL for v in want_n])   # Python integers: exact, non-negative
    np.testing.assert_array_equal(idx, exact_mod)
    assert np.all(np.abs(y) <= 0.5)
    # y is exact: n + y reproduces tu
    np.testing.assert_array_equal(n + y, tu)
    # where an int32 conversion would have clamped the index is now right
    big = np.abs(tu) > 2.0 ** 31
    assert big.sum() > 2000


def test_phase_limit_keeps_table_units_below_2_51():
    assert PHASE_LIMIT * PH_TBL < 2.0 ** 51
    idx, n, y = kernel_index(np.array([PHASE_LIMIT * PH_TBL - 0.75, -PHASE_LIMIT * PH_TBL + 0.25]))
    np.testing.assert_array_equal(n + y, [PHASE_LIMIT * PH_TBL - 0.75, -PHASE_LIMIT * PH_TBL + 0.25])
