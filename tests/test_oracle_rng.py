"""Statistical pins of the oracle's Philox4x32-10 stream and its conversions."""
import numpy as np
import pytest
from scipy import stats

from oracle import oracle as O


def words(seed, stream, n, step=0, d=0):
    out = np.zeros((n, 4), np.uint32)
    for e in range(n):
        out[e] = O.draw(seed, stream, e, step, d)
    return out


def test_uniform_conversion_bounds():
    assert O.uniform(0) == pytest.approx(0.5 / 2 ** 32, rel=1e-15)
    assert 0.0 < O.uniform(0) < O.uniform(1) < O.uniform(2 ** 32 - 1) < 1.0
    assert O.uniform(2 ** 31) == 0.5 + 0.5 / 2 ** 32


def test_index_conversion_exact():
    assert O.index(0, 7) == 0
    assert O.index(2 ** 32 - 1, 7) == 6
    # floor(w * n / 2^32) for a few hand values
    for w, n in [(123456789, 1000), (2 ** 31, 3), (3 * 2 ** 30, 4), (2 ** 32 - 1, 1)]:
        assert O.index(w, n) == (w * n) >> 32


def test_philox_uniformity_chi2():
    w = words(12345, 0, 20000).reshape(-1)
    hist = np.bincount((w >> 24).astype(np.int64), minlength=256)
    chi2, p = stats.chisquare(hist)
    assert p > 1e-4
    # every bit is fair
    bits = ((w[:, None] >> np.arange(32, dtype=np.uint32)) & 1).mean(axis=0)
    assert np.all(np.abs(bits - 0.5) < 5 * 0.5 / np.sqrt(len(w)))


def test_philox_serial_independence():
    w = words(7, 1, 20000).astype(np.float64) / 2 ** 32
    for lag_words in (w[:, 0], w[:, 1], w[:, 2], w[:, 3]):
        r = np.corrcoef(lag_words[:-1], lag_words[1:])[0, 1]
        assert abs(r) < 4 / np.sqrt(len(lag_words))
    r = np.corrcoef(w[:, 0], w[:, 3])[0, 1]
    assert abs(r) < 4 / np.sqrt(len(w))


def test_philox_avalanche():
    # flipping one counter or key bit flips about half of the 128 output bits
    rng = np.random.default_rng(3)
    flips = []
    for _ in range(300):
        ctr = [int(x) for x in rng.integers(0, 2 ** 32, 4)]
        key = [int(x) for x in rng.integers(0, 2 ** 32, 2)]
        a = O.philox(ctr, key)
        b_ctr = list(ctr)
        word, bit = int(rng.integers(4)), int(rng.integers(32))
        b_ctr[word] ^= 1 << bit
        b = O.philox(b_ctr, key)
        flips.append(sum(bin(x ^ y).count("1") for x, y in zip(a, b)))
        k2 = list(key)
        k2[int(rng.integers(2))] ^= 1 << int(rng.integers(32))
        c = O.philox(ctr, k2)
        flips.append(sum(bin(x ^ y).count("1") for x, y in zip(a, c)))
    assert abs(np.mean(flips) - 64) < 1.5


def test_streams_steps_and_seeds_are_distinct():
    base = O.draw(1, 0, 5, 3, 9)
    assert O.draw(2, 0, 5, 3, 9) != base
    assert O.draw(1, 1, 5, 3, 9) != base
    assert O.draw(1, 0, 6, 3, 9) != base
    assert O.draw(1, 0, 5, 4, 9) != base
    assert O.draw(1, 0, 5, 3, 10) != base
    assert O.draw(1, 0, 5, 3, 9) == base
    # high entity bits reach the counter (ids above 2^32)
    assert O.draw(1, 0, 5 + (1 << 32), 3, 9) != base


def _kat_vectors():
    """Rows of tests/golden/philox4x32_10_kat.txt: (ctr[4], key[2], out[4])."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")
    rows = []
    with open(path) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            lhs, rhs = line.split("->")
            a = [int(x, 16) for x in lhs.split()]
            rows.append((a[:4], a[4:6], [int(x, 16) for x in rhs.split()]))
    return rows


def kat_as_draw(ctr, key):
    """The (seed, stream, entity, step, draw) whose counter layout gives ctr, key:
    ctr = (entity bits 0-31, entity bits 32-59 | stream << 28, step, draw), key = seed."""
    stream = ctr[1] >> 28
    entity = ((ctr[1] & 0x0FFFFFFF) << 32) | ctr[0]
    return key[0] | (key[1] << 32), stream, entity, ctr[2], ctr[3]


def test_philox_known_answers():
    rows = _kat_vectors()
    assert len(rows) == 3
    for ctr, key, out in rows:
        assert list(O.philox(ctr, key)) == out
        # the same words through the (seed, stream, entity, step, draw) counter layout
        assert list(O.draw(*kat_as_draw(ctr, key))) == out
