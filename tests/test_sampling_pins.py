"""Pins of the oracle's candidate sampler (row "candidate controls" of the hot
path: the paper draws the samples on the device with a counter-based
generator, section "Real-Time Implementation").

The generator bits are pinned against numpy's own, independent implementation
of Philox4x64-10 (numpy.random.Philox); the maps from bits to controls are
pinned by their distributions (Kolmogorov-Smirnov against the exact uniform
and normal laws), their moments and independence, and by the nominal and
keep-nominal special cases."""
import numpy as np
import pytest
from scipy import stats

import oracle

MASK = (1 << 64) - 1


def numpy_block(counter, key):
    """Philox4x64-10 output block at `counter` from numpy's generator. numpy
    advances its 256-bit counter before producing a block, so it is seeded
    with counter - 1."""
    c = sum(int(w) << (64 * i) for i, w in enumerate(counter))
    c = (c - 1) % (1 << 256)
    words = np.array([(c >> (64 * i)) & MASK for i in range(4)], dtype=np.uint64)
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=words)
    return bg.random_raw(4).astype(np.uint64)


@pytest.mark.parametrize("counter,key", [
    ([0, 0, 0, 0], [0, 0]),
    ([1, 0, 0, 0], [0, 0]),
    ([7, 3, 0, 0], [123, 456]),
    ([MASK, MASK, MASK, MASK], [MASK, MASK]),
    ([0x243F6A8885A308D3, 0x13198A2E03707344, 0xA4093822299F31D0, 0x082EFA98EC4E6C89],
     [0x452821E638D01377, 0xBE5466CF34E90C6C]),
    ([4095, 24, 0, 0], [2603, 20525]),
])
def test_philox_matches_numpy(counter, key):
    got = oracle.philox4x64(counter, key)
    assert np.array_equal(got, numpy_block(counter, key))


def test_sample_layout_uses_counter_k_n_div_4_and_word_n_mod_4():
    seed, stream, K, N = 77, 5, 6, 9
    u = oracle.sample_controls(oracle.SAMPLE_UNIFORM, seed, stream, [1.0, 1.0], K, N)
    for k in range(K):
        for n in range(N):
            w = int(numpy_block([k, n // 4, 0, 0], [seed, stream])[n % 4])
            a, b = w >> 40, (w >> 16) & 0xFFFFFF
            # 2x - 1 with x = a 2^-24 is exact in double; so is the comparison
            assert u[n, 0, k] == 2.0 * (a / 2.0**24) - 1.0
            assert u[n, 1, k] == 2.0 * (b / 2.0**24) - 1.0


def test_uniform_law_and_range():
    s = [1.0, 0.25]
    u = oracle.sample_controls(oracle.SAMPLE_UNIFORM, 11, 0, s, 4000, 16)
    for c in range(2):
        x = u[:, c, :].ravel()
        assert x.min() >= -s[c] and x.max() < s[c]
        assert stats.kstest(x, stats.uniform(loc=-s[c], scale=2 * s[c]).cdf).pvalue > 1e-3
    # the two channels and neighbouring intervals/candidates are uncorrelated
    assert abs(np.corrcoef(u[:, 0, :].ravel(), u[:, 1, :].ravel())[0, 1]) < 0.02
    assert abs(np.corrcoef(u[:-1, 0, :].ravel(), u[1:, 0, :].ravel())[0, 1]) < 0.02
    assert abs(np.corrcoef(u[:, 0, :-1].ravel(), u[:, 0, 1:].ravel())[0, 1]) < 0.02


def test_gaussian_law_moments_and_independence():
    s = [0.1, 0.2]
    u = oracle.sample_controls(oracle.SAMPLE_GAUSSIAN, 3, 1, s, 4000, 20)
    for c in range(2):
        x = u[:, c, :].ravel()
        assert stats.kstest(x, stats.norm(scale=s[c]).cdf).pvalue > 1e-3
        assert abs(x.mean()) < 4 * s[c] / np.sqrt(x.size)
        assert abs(x.std() / s[c] - 1) < 0.02
    # Box-Muller pairs are independent normals, not merely uncorrelated marginals
    z0 = u[:, 0, :].ravel() / s[0]
    z1 = u[:, 1, :].ravel() / s[1]
    assert abs(np.corrcoef(z0, z1)[0, 1]) < 0.02
    assert abs(np.corrcoef(z0**2, z1**2)[0, 1]) < 0.03
    r2 = z0**2 + z1**2
    assert stats.kstest(r2, stats.chi2(df=2).cdf).pvalue > 1e-3


def test_streams_and_seeds_give_distinct_samples():
    a = oracle.sample_controls(oracle.SAMPLE_GAUSSIAN, 3, 1, [1, 1], 64, 8)
    b = oracle.sample_controls(oracle.SAMPLE_GAUSSIAN, 3, 2, [1, 1], 64, 8)
    c = oracle.sample_controls(oracle.SAMPLE_GAUSSIAN, 4, 1, [1, 1], 64, 8)
    assert not np.any(a == b) and not np.any(a == c)


def test_nominal_offset_and_keep_nominal():
    K, N = 32, 10
    rng = np.random.default_rng(0)
    nom = rng.normal(size=(N, 2)).astype(np.float32)
    base = oracle.sample_controls(oracle.SAMPLE_GAUSSIAN, 9, 0, [0.1, 0.2], K, N)
    off = oracle.sample_controls(oracle.SAMPLE_GAUSSIAN, 9, 0, [0.1, 0.2], K, N, nominal=nom)
    assert np.allclose(off - base, nom.astype(np.float64)[:, :, None], rtol=0, atol=1e-12)
    keep = oracle.sample_controls(oracle.SAMPLE_GAUSSIAN, 9, 0, [0.1, 0.2], K, N, nominal=nom,
                                  keep_nominal=True)
    assert np.array_equal(keep[:, :, 0], nom.astype(np.float64))
    assert np.array_equal(keep[:, :, 1:], off[:, :, 1:])
    # zero scale reproduces the nominal for every candidate
    z = oracle.sample_controls(oracle.SAMPLE_UNIFORM, 9, 0, [0.0, 0.0], K, N, nominal=nom)
    assert np.array_equal(z, np.repeat(nom.astype(np.float64)[:, :, None], K, axis=2))


def test_invalid_arguments_are_rejected():
    with pytest.raises(ValueError):
        oracle.sample_controls(2, 0, 0, [1, 1], 4, 4)
    with pytest.raises(ValueError):
        oracle.sample_controls(0, 0, 0, [1, 1], 0, 4)
