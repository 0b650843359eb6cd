"""The float32 bit-pattern facts the kernels rely on (host logic, no GPU).

The eager relaxation takes min(d, s) on the 32-bit patterns of two float32
values instead of selecting on the comparison s < d, and the direct-copy
kernels compare operand panels the same way.  That gives the same bits
exactly when both values are non-negative (+0 .. +inf) and neither is NaN or
-0: the solver normalises its input that way (NaN becomes +inf, -0 becomes
+0), and a sum of two such values is again such a value.
"""
import numpy as np

F32_INF = np.float32(np.inf)


def _nonneg_f32(rng, count):
    """Non-negative float32 values over every exponent: zero, subnormals,
    normals, the largest finite value and +inf, plus exact duplicates."""
    bits = rng.integers(0, 0x7F800000, size=count, dtype=np.uint32)
    v = bits.view(np.float32).copy()
    v[: count // 16] = 0.0
    v[count // 16: count // 8] = F32_INF
    v[count // 8: count // 8 + 8] = np.finfo(np.float32).max
    v[count // 8 + 8: count // 8 + 16] = np.finfo(np.float32).smallest_subnormal
    rng.shuffle(v)
    return v


def test_min_on_bits_equals_strict_select():
    rng = np.random.default_rng(11)
    d = _nonneg_f32(rng, 1 << 16)
    s = _nonneg_f32(rng, 1 << 16)
    s[::7] = d[::7]                                      # ties
    select = np.where(s < d, s, d)
    by_bits = np.minimum(d.view(np.uint32), s.view(np.uint32)).view(np.float32)
    np.testing.assert_array_equal(by_bits.view(np.uint32), select.view(np.uint32))


def test_sums_stay_non_negative_and_ordered():
    """a + b of two normalised values is never NaN or -0, so a relaxation's
    sum can enter the next minimum on bits."""
    rng = np.random.default_rng(12)
    a = _nonneg_f32(rng, 1 << 16)
    b = _nonneg_f32(rng, 1 << 16)
    with np.errstate(over="ignore"):
        s = a + b
    assert s.dtype == np.float32
    assert not np.isnan(s).any()
    assert not (np.signbit(s)).any()
    # bit order = value order on the sums too
    order_bits = np.argsort(s.view(np.uint32), kind="stable")
    order_vals = np.argsort(s, kind="stable")
    np.testing.assert_array_equal(s[order_bits], s[order_vals])


def test_negative_zero_would_break_it():
    """Why the input is normalised: -0 (sign bit set) is the largest pattern
    on bits although it equals +0, so a minimum on bits would keep +0 where
    the select keeps d = -0 -- different bits."""
    d = np.array([-0.0], np.float32)
    s = np.array([0.0], np.float32)
    select = np.where(s < d, s, d)
    by_bits = np.minimum(d.view(np.uint32), s.view(np.uint32)).view(np.float32)
    assert select.view(np.uint32)[0] != by_bits.view(np.uint32)[0]
