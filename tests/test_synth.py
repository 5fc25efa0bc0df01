"""Pins for the seeded input generator (CPU only)."""
import os

import numpy as np

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
GAMMA = np.uint64(0x9E3779B97F4A7C15)
TGAMMA = 0xD1B54A32D192ED03


def _np_splitmix(seed_t, ks):
    """SplitMix64's mix function written out with numpy uint64 wrap-around."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed_t) + (ks.astype(np.uint64) + np.uint64(1)) * GAMMA
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def test_published_vector():
    want = [int(l) for l in open(os.path.join(GOLDEN, "splitmix64_seed1234567.txt"))
            if l.strip() and not l.startswith("#")]
    got = synth.raw(1234567 ^ TGAMMA, 0, 5)
    assert [int(v) for v in got] == want


def test_counter_streams_match_numpy_twin():
    for seed, t in [(1, 0), (2, 2), (3, 7)]:
        ks = np.arange(1000, 3000)
        seed_t = (seed ^ ((t + 1) * TGAMMA)) & 0xFFFFFFFFFFFFFFFF
        assert np.array_equal(synth.raw(seed, t, 2000, start=1000), _np_splitmix(seed_t, ks))


def test_ranges_are_independent():
    a = synth.fill(2, 1, 5000, "f32")
    b = synth.fill(2, 1, 3000, "f32", start=2000)
    assert np.array_equal(a[2000:], b)


def test_uniform_definition_and_range():
    r = synth.raw(1, 0, 4096)
    want = 2.0 * ((r >> np.uint64(11)).astype(np.float64) * 2.0 ** -53) - 1.0
    got = synth.fill_f64(1, 0, 4096)
    assert np.array_equal(got, want)
    assert got.min() >= -1.0 and got.max() < 1.0
    assert np.array_equal(synth.fill(1, 0, 4096, "f32"), want.astype(np.float32))


def test_uint31():
    r = synth.raw(1, 2, 4096)
    assert np.array_equal(synth.fill(1, 2, 4096, "u32", "uint31"),
                          (r >> np.uint64(33)).astype(np.uint32))


def test_f16_rounding_is_numpy_nearest_even():
    v = synth.fill_f64(3, 0, 50000, "lognormal", 3.0)
    h, sat = synth.fill(3, 0, 50000, "f16", "lognormal", 3.0, return_saturations=True)
    want = v.astype(np.float16)  # numpy rounds double -> half directly, nearest-even
    big = np.abs(v) > 65504
    want[big] = np.copysign(np.float16(65504), v[big])
    assert sat == int(big.sum())
    # numpy turns |v| >= 65520 into inf; the generator saturates instead
    assert np.array_equal(h.view(np.uint16), want.view(np.uint16))


def _bf16_vals(bits):
    return synth.bf16_to_f64(bits)


def test_bf16_rounding_is_nearest_even():
    v = np.concatenate([synth.fill_f64(3, 1, 20000),
                        synth.fill_f64(3, 1, 20000, "lognormal", 3.0)])
    bits = np.concatenate([synth.fill(3, 1, 20000, "bf16"),
                           synth.fill(3, 1, 20000, "bf16", "lognormal", 3.0)])
    r = _bf16_vals(bits)
    up = _bf16_vals((bits.astype(np.int32) + 1).astype(np.uint16))
    dn = _bf16_vals((bits.astype(np.int32) - 1).astype(np.uint16))
    # the chosen value is at least as close as both neighbours ...
    e = np.abs(v - r)
    assert np.all(e <= np.abs(v - up)) and np.all(e <= np.abs(v - dn))
    # ... and on a tie the mantissa is even
    tie = (e == np.abs(v - up)) | (e == np.abs(v - dn))
    assert np.all((bits[tie] & 1) == 0)


def test_bf16_exact_ties():
    # 1 + 2^-8 is halfway between bf16 neighbours 1 and 1 + 2^-7: even is 1.
    # Written through the "ones" distribution, which rounds its parameter.
    for val, want in [(1.0 + 2 ** -8, 0x3F80), (1.0 + 3 * 2 ** -8, 0x3F82),
                      (-(1.0 + 2 ** -8), 0xBF80), (2.0 ** -130, None)]:
        b = synth.fill(0, 0, 1, "bf16", "ones", val)[0]
        if want is not None:
            assert b == want
        else:  # subnormal bf16 keeps its value exactly (2^-130 = 2^-133 * 8)
            assert _bf16_vals(np.array([b], np.uint16))[0] == val


def test_lognormal_heavy_tail_shape():
    v = synth.fill_f64(3, 2, 200000, "lognormal", 3.0)
    g = np.log(np.abs(v)) / 3.0
    assert abs(g.mean()) < 0.01 and abs(g.std() - 1.0) < 0.01
    assert 0.45 < (v > 0).mean() < 0.55


def test_uniform12():
    r = synth.raw(3, 5, 2000)
    want = 1.0 + (r >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    assert np.array_equal(synth.fill_f64(3, 5, 2000, "uniform12"), want)
    assert want.min() >= 1.0 and want.max() < 2.0
