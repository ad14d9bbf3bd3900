"""Pin: the oracle's Philox4x64-10 equals numpy's independent implementation of
the same published generator (numpy.random.Philox), bit for bit."""
import numpy as np

import oracle


def _numpy_philox(ctr, key):
    c = sum(int(x) << (64 * i) for i, x in enumerate(ctr))
    k = int(key[0]) | (int(key[1]) << 64)
    # numpy increments its 256-bit counter before producing a block
    bg = np.random.Philox(counter=(c - 1) % (1 << 256), key=k)
    return bg.random_raw(4)


def test_philox_matches_numpy():
    rng = np.random.default_rng(7)
    ctrs = rng.integers(0, np.iinfo(np.uint64).max, size=(64, 4), dtype=np.uint64, endpoint=True)
    ctrs[0] = 0
    ctrs[1] = [1, 0, 0, 0]
    ctrs[2] = np.iinfo(np.uint64).max
    for key in ([0, 0], [123456789, 0], [np.iinfo(np.uint64).max, 42]):
        key = np.array(key, dtype=np.uint64)
        got = oracle.philox4x64(ctrs, key)
        for i in range(len(ctrs)):
            assert np.array_equal(got[i], _numpy_philox(ctrs[i], key)), (i, key)


def test_uniforms_are_uniform():
    # chi-square of the 24-bit uniforms drawn from consecutive counters
    n = 1 << 16
    ctr = np.zeros((n, 4), dtype=np.uint64)
    ctr[:, 0] = np.arange(n)
    r = oracle.philox4x64(ctr, np.array([5, 0], dtype=np.uint64))
    u = ((r[:, 0] & np.uint64(0xFFFFFFFF)) >> np.uint64(8)).astype(np.float64) / 2 ** 24
    h, _ = np.histogram(u, bins=64, range=(0, 1))
    e = n / 64
    chi2 = ((h - e) ** 2 / e).sum()
    assert chi2 < 120  # 63 dof: p ~ 1e-5
