"""The bfloat16 write path's rounding arithmetic, emulated bit by bit in numpy (no GPU).

A cold row unit is stored as SR(old + inc): stochastic rounding to bfloat16 by adding 16
random bits below the kept half of the binary32 pattern and truncating.  A hot row unit
instead receives, by a packed bfloat16 atomic add, the increment SR(old + inc) - old
(rounded to nearest even to bfloat16).  These tests pin what the hot path rests on, over
many random operands:
  * while old and SR(old + inc) are within a factor of two of each other (so whenever
    |inc| <= |old| / 2) the increment is exactly representable (Sterbenz) and adding it to
    old gives SR(old + inc) bit for bit;
  * for any operands the result is within one bfloat16 spacing of SR(old + inc);
  * SR is unbiased, E[SR(x)] = x, so increments below half a spacing survive on average.
"""
import numpy as np


def f32_to_bf16_sr(x: np.ndarray, rnd16: np.ndarray) -> np.ndarray:
    u = x.astype(np.float32).view(np.uint32).astype(np.uint64)
    return ((u + (rnd16.astype(np.uint64) & 0xFFFF)) >> 16).astype(np.uint32)


def f32_to_bf16_rne(x: np.ndarray) -> np.ndarray:
    u = x.astype(np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    return ((u + 0x7FFF + lsb) >> 16).astype(np.uint32)


def bf16_to_f32(h: np.ndarray) -> np.ndarray:
    return (h.astype(np.uint32) << 16).view(np.float32)


def _operands(n, rng):
    old = bf16_to_f32(f32_to_bf16_rne(rng.standard_normal(n).astype(np.float32) * np.float32(0.3)))
    rel = np.exp(rng.uniform(np.log(1e-6), np.log(0.5), n)).astype(np.float32)
    inc = (old * rel * rng.choice([-1.0, 1.0], n)).astype(np.float32)
    rnd = rng.integers(0, 1 << 16, n, dtype=np.uint32)
    return old, inc, rnd


def test_sr_increment_is_representable_and_lands_on_sr():
    rng = np.random.default_rng(2604)
    old, inc, rnd = _operands(1_000_000, rng)  # |inc| <= |old| / 2
    target = f32_to_bf16_sr(old + inc, rnd)                     # what a cold store writes
    delta = bf16_to_f32(target) - old                            # binary32, exact
    delta_bf = f32_to_bf16_rne(delta)                            # what the atomic adds
    assert np.array_equal(bf16_to_f32(delta_bf), delta)         # representable
    landed = f32_to_bf16_rne(old + bf16_to_f32(delta_bf))        # the atomic's sum, rounded
    assert np.array_equal(landed, target)                        # = SR(old + inc), bitwise


def test_increments_below_half_a_spacing_survive_on_average():
    """Rounding to nearest would drop every such increment; stochastic rounding keeps its
    mean: over 2^16 equally spaced random words E[SR(x)] equals x up to binary32 rounding."""
    old = np.float32(0.3)
    spacing = np.float32(2.0 ** -9)   # bfloat16 spacing of [0.25, 0.5)
    old = bf16_to_f32(f32_to_bf16_rne(np.array([old])))[0]
    for frac in (0.01, 0.1, 0.37):
        inc = np.float32(frac) * spacing
        x = np.full(1 << 16, old + inc, dtype=np.float32)
        rnd = np.arange(1 << 16, dtype=np.uint32)
        mean = bf16_to_f32(f32_to_bf16_sr(x, rnd)).astype(np.float64).mean()
        assert abs(mean - float(np.float32(old + inc))) < 1e-9
        assert f32_to_bf16_rne(np.array([old + inc]))[0] == f32_to_bf16_rne(np.array([old]))[0]


def test_large_increments_land_within_one_spacing():
    """|inc| up to 100 |old| (rows near zero): the increment may need rounding, and the
    result then differs from SR(old + inc) by at most one bfloat16 spacing of the larger of
    the two magnitudes."""
    rng = np.random.default_rng(7)
    n = 1_000_000
    old = bf16_to_f32(f32_to_bf16_rne(rng.standard_normal(n).astype(np.float32) * np.float32(0.01)))
    rel = np.exp(rng.uniform(np.log(1e-6), np.log(100.0), n)).astype(np.float32)
    inc = (np.abs(old) * rel * rng.choice([-1.0, 1.0], n)).astype(np.float32)
    rnd = rng.integers(0, 1 << 16, n, dtype=np.uint32)
    target = bf16_to_f32(f32_to_bf16_sr(old + inc, rnd)).astype(np.float64)
    delta = bf16_to_f32(f32_to_bf16_sr(old + inc, rnd)) - old
    landed = bf16_to_f32(f32_to_bf16_rne(old + bf16_to_f32(f32_to_bf16_rne(delta)))).astype(np.float64)
    mag = np.maximum(np.abs(target), np.abs(old.astype(np.float64)))
    spacing = 2.0 ** (np.floor(np.log2(np.where(mag > 0, mag, 1.0))) - 7)
    assert np.all(np.abs(landed - target) <= spacing)
    small = rel <= 0.5
    assert np.array_equal(landed[small], target[small])
