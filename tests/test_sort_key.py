"""The fixed-point sort key of the neighbour selection, emulated on the CPU.

The step kernel orders a lane's candidate entries with a sorting network over
32-bit words: the entry's FP32 key f (the FP64 squared distance rounded to
FP32) scaled to 26 bits of the counted squared radius r2c, above a 6-bit
buffer slot,

    q = min(trunc(f * RN32(2^26 / r2c)), 2^26 - 1),   word = q << 6 | slot,

with the FP32 product rounded once.  The exact-kNN contract (each agent's k
nearest, Sec. 3's nearby agents, ties by index) needs the word to be
non-decreasing in the key: then distinct words are in key order and equal
words go to the exact insertion pass.  These tests evaluate the formula in
numpy FP32 for keys up to r2c, including the last few 1e-8 below it where
the FP32 product reaches 2^26 (a clamp written as an FP32 minimum against
2^26 - 1 cannot hold there: that value rounds to 2^26 in FP32, and the
shift then wraps the word to the slot alone).
"""
import numpy as np
import pytest

TWO26 = np.float32(67108864.0)
QMAX = (1 << 26) - 1


def packed_word(key, r2c, slot=0):
    """The kernel's word for FP64 keys `key` (array) below r2c."""
    fk = np.asarray(key, np.float64).astype(np.float32)
    qscale = TWO26 / np.float32(r2c)
    prod = (fk * qscale).astype(np.float32)   # one FP32 rounding
    q = np.minimum(prod.astype(np.float64).astype(np.uint64), QMAX)  # truncation, integer clamp
    return ((q << 6) | slot) & 0xFFFFFFFF


def float_clamped_word(key, r2c, slot=0):
    """A clamp in FP32 instead: min(f * scale, float(2^26 - 1)), shifted."""
    fk = np.asarray(key, np.float64).astype(np.float32)
    prod = np.minimum((fk * (TWO26 / np.float32(r2c))).astype(np.float32),
                      np.float32(67108863.0))
    q = prod.astype(np.float64).astype(np.uint64)
    return ((q << 6) | slot) & 0xFFFFFFFF


# squared radii the kernel counts against: R_n^2 of the workloads (3, 4.5 and
# 5 m) and kept-distance circles (d_K + margin)^2 of arbitrary size
R2C = [9.0, 20.25, 25.0, 16.0, 1.476, 3.516, 0.36, 123.456789] + \
      list(np.random.default_rng(5).uniform(0.05, 30.0, 24))


@pytest.mark.parametrize("r2c", R2C)
def test_word_non_decreasing_up_to_the_counted_radius(r2c):
    rng = np.random.default_rng(int(r2c * 1000) % 2**31)
    near = r2c * (1.0 - rng.uniform(0.0, 1e-6, 20000))
    edge = r2c * (1.0 - np.logspace(-16, -6, 4000))
    spread = rng.uniform(0.0, r2c, 20000)
    key = np.sort(np.concatenate([near, edge, spread, [0.0]]))
    key = key[key < r2c]
    w = packed_word(key, r2c)
    assert (np.diff(w.astype(np.int64)) >= 0).all()
    assert w.max() <= QMAX << 6
    # the 26-bit key spans the range: zero at distance zero, close to the top
    # just below r2c
    assert packed_word([0.0], r2c)[0] == 0
    assert packed_word([r2c * (1 - 1e-12)], r2c)[0] >> 6 >= QMAX - 4


def test_every_fp32_key_below_the_radius():
    # all FP32 keys from 0.999 r2c up to the largest below r2c, one by one
    for r2c in (9.0, 25.0, 1.476):
        top = np.float32(r2c)
        lo = np.float32(r2c * 0.999)
        keys = np.arange(lo.view(np.int32), top.view(np.int32) + 1, dtype=np.int32).view(np.float32)
        keys = keys.astype(np.float64)
        keys = np.minimum(keys, np.nextafter(r2c, 0.0))  # FP64 keys round to these FP32 values
        w = packed_word(keys, r2c)
        assert (np.diff(w.astype(np.int64)) >= 0).all(), r2c


def test_float_clamp_wraps_at_the_radius():
    # the reason for the integer clamp: keys within about 1e-8 below r2c give
    # an FP32 product of exactly 2^26, which a float clamp keeps, and the
    # shifted word wraps to 0 -- the farthest candidate would sort first
    for r2c in (9.0, 25.0, 20.25, 1.476, 3.516):
        key = np.array([r2c * (1 - 1e-8), r2c * 0.5])
        bad = float_clamped_word(key, r2c)
        assert bad[0] == 0 and bad[1] > 0, r2c
        good = packed_word(key, r2c)
        assert good[0] > good[1], r2c
