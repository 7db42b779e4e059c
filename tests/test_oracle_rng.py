"""Pins of the oracle's SplitMix64 (Steele, Lea & Flood 2014)."""
import numpy as np

from oracle import rng


def test_splitmix64_published_first_output():
    # First output of the reference SplitMix64 seeded with 0 (state += GAMMA,
    # then mix): 0xE220A8397B1DCDAF.
    assert rng.mix_int(0 + rng.GAMMA) == 0xE220A8397B1DCDAF


def test_vectorised_mix_matches_integer_mix():
    rs = np.random.default_rng(0)
    xs = rs.integers(0, 2**63, size=64, dtype=np.uint64)
    got = rng.mix_u64(xs)
    for x, g in zip(xs, got):
        assert int(g) == rng.mix_int(int(x))


def test_uniform_range_and_mean():
    u = rng.uniform(rng.stream_key(7, 0), np.arange(200000, dtype=np.uint64))
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 5e-3
    # stream origin is the counter -1 state: counter c uses state key + (c+1) GAMMA
    k = rng.stream_key(7, 0)
    assert rng.uniform(k, np.array([3], np.uint64))[0] == \
        (rng.mix_int(k + 4 * rng.GAMMA) >> 11) * 2.0 ** -53
