"""Pins of the oracle's counter-based noise.

The Langevin noise of Appendix A (delta-correlated, variance 2 gamma kT) is
drawn from Philox4x32-10 (Salmon et al., SC'11) keyed by the seed, with the
counter (nucleotide, stream/call, step).  The oracle's round structure is also
built on 64-bit words (Philox4x64-10) and pinned bit for bit against numpy's
independent implementation of that generator; the Box-Muller normals are
checked against the normal distribution.
"""
import numpy as np
import pytest
from scipy import stats


@pytest.mark.parametrize("ctr,key", [
    ([0, 0, 0, 0], [0, 0]),
    ([1, 2, 3, 4], [5, 6]),
    ([2**64 - 2, 7, 2**63, 11], [0xDEADBEEFCAFEF00D, 0x0123456789ABCDEF]),
    ([123456789, 0, 0, 2**64 - 1], [2**64 - 1, 2**64 - 1]),
])
def test_philox4x64_matches_numpy(orc, ctr, key):
    """numpy's Philox(counter=c, key=k) first increments the 256-bit counter
    (lowest word first) and then emits the four words of Philox4x64-10(c+1, k)."""
    bg = np.random.Philox(counter=np.array(ctr, dtype=np.uint64), key=np.array(key, dtype=np.uint64))
    want = bg.random_raw(4)
    c_int = (sum(int(x) << (64 * k) for k, x in enumerate(ctr)) + 1) % 2**256
    c = [(c_int >> (64 * k)) & (2**64 - 1) for k in range(4)]
    got = orc.philox4x64(np.array(c, dtype=np.uint64), np.array(key, dtype=np.uint64))
    assert np.array_equal(got, want)


def test_philox4x32_is_keyed_and_counter_sensitive(orc):
    """Every input word changes every output word (avalanche), and outputs of
    distinct counters are distinct."""
    base = orc.philox4x32([1, 2, 3, 4], [5, 6])
    for k in range(4):
        c = [1, 2, 3, 4]
        c[k] ^= 1
        o = orc.philox4x32(c, [5, 6])
        assert np.all(o != base)
    for k in range(2):
        key = [5, 6]
        key[k] ^= 1
        assert np.all(orc.philox4x32([1, 2, 3, 4], key) != base)
    outs = {tuple(orc.philox4x32([i, 0, 0, 0], [9, 9])) for i in range(2000)}
    assert len(outs) == 2000


def test_philox4x32_bits_uniform(orc):
    """Output words are uniform on [0, 2^32): a chi-square test on 64 bins and
    a test of each bit's frequency."""
    w = np.concatenate([orc.philox4x32([i, 7, 3, 0], [1, 2]) for i in range(20000)]).astype(np.uint64)
    counts = np.bincount((w >> 26).astype(np.int64), minlength=64)
    assert stats.chisquare(counts).pvalue > 1e-4
    for b in range(32):
        f = ((w >> b) & 1).mean()
        assert abs(f - 0.5) < 5 * 0.5 / np.sqrt(len(w))


def test_gaussian_noise_is_standard_normal(orc):
    xi = np.concatenate([orc.noise(seed=42, noise_kind=0, step_=s, nt_id=i)
                         for s in range(40) for i in range(500)])
    assert abs(xi.mean()) < 5 / np.sqrt(len(xi))
    assert abs(xi.var() - 1.0) < 5 * np.sqrt(2.0 / len(xi))
    assert stats.kstest(xi, "norm").pvalue > 1e-4
    # components are uncorrelated
    X = xi.reshape(-1, 6)
    C = np.corrcoef(X.T)
    assert np.abs(C - np.eye(6)).max() < 5 / np.sqrt(X.shape[0])


def test_uniform_noise_matches_variance(orc):
    xi = np.concatenate([orc.noise(seed=3, noise_kind=1, step_=s, nt_id=i)
                         for s in range(20) for i in range(500)])
    assert np.abs(xi).max() <= np.sqrt(3.0)
    assert abs(xi.var() - 1.0) < 5 * np.sqrt(0.8 / len(xi))
    assert stats.kstest(xi, "uniform", args=(-np.sqrt(3), 2 * np.sqrt(3))).pvalue > 1e-4


def test_noise_is_a_function_of_seed_step_and_id(orc):
    a = orc.noise(5, 0, 17, 3)
    assert np.array_equal(a, orc.noise(5, 0, 17, 3))
    assert not np.array_equal(a, orc.noise(6, 0, 17, 3))
    assert not np.array_equal(a, orc.noise(5, 0, 18, 3))
    assert not np.array_equal(a, orc.noise(5, 0, 17, 4))
    assert not np.array_equal(a, orc.noise(5, 0, 17, 3, stream=1))
    # steps beyond 2^32 use the high counter word
    assert not np.array_equal(orc.noise(5, 0, 1, 3), orc.noise(5, 0, 1 + 2**32, 3))
