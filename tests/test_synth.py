"""The seeded input generator (paper_1903_08882_amd/synth.py) against the
published definition of splitmix64: from state 0 the generator's first
outputs are 0xe220a8397b1dcdaf, 0x6e789e6aa1b965f4, 0x06c45d188009454f (the
reference sequence of Vigna's splitmix64.c, the finaliser of Steele, Lea &
Flood's SplittableRandom); and the properties the tests rely on: the same
(seed, stream) gives the same numbers, different streams differ, values lie
in [-1, 1) on the 2^-52 grid, and the rest state carries noise in T only."""
import numpy as np

from paper_1903_08882_amd import synth


def test_splitmix64_reproduces_the_published_sequence():
    g = np.uint64(0x9E3779B97F4A7C15)
    with np.errstate(over="ignore"):
        out = [int(synth.splitmix64(np.uint64(k) * g)) for k in range(3)]
    assert out == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_uniform_is_deterministic_in_range_and_stream_separated():
    a = synth.uniform(synth.SEED0, 0, 100_000)
    assert np.array_equal(a, synth.uniform(synth.SEED0, 0, 100_000))
    assert a.min() >= -1.0 and a.max() < 1.0
    assert np.all(((a + 1.0) * 2.0 ** 52) % 1.0 == 0.0)          # top 53 bits, exactly
    assert abs(a.mean()) < 0.01 and abs(np.mean(a * a) - 1.0 / 3.0) < 0.01
    b = synth.uniform(synth.SEED0, 1, 100_000)
    assert abs(np.corrcoef(a, b)[0, 1]) < 0.01
    assert not np.array_equal(a[:1000], synth.uniform(synth.SEED0 + 1, 0, 1000))


def test_rest_state_has_noise_in_temperature_only():
    f = synth.rest_with_noise(9)
    assert f.shape == (4, 9, 9, 9)
    assert not f[:3].any() and 0.0 < np.abs(f[3]).max() < 1e-3
    assert np.array_equal(f[3], 1e-3 * synth.uniform(synth.SEED0, 0, 9 ** 3).reshape(9, 9, 9))
