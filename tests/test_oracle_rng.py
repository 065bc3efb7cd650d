"""Pins of the oracle's random numbers.  The paper only asks for independent
unit Gaussians per mode and step (Sec. IV).  The generator is Philox4x32-10
(Salmon et al., SC'11) with 24-bit uniforms and Box-Muller pairs.  The
Philox output is pinned to the published generator's known-answer vectors
(golden fixture `philox_kat.txt`), and bit for bit to an independent
pure-Python implementation over random counters and keys; the 24-bit
chunking and the normals are pinned by the same Python twin, by statistical
tests of the bits, and by the normals' moments and a Kolmogorov-Smirnov
test against N(0, 1)."""
import numpy as np
import pytest
from scipy import stats

import oracle
from tests import lbtheory as th


def load_philox_kat():
    """[(counter[4], key[2], output[4])] from the known-answer fixture."""
    rows = []
    with open(th.os.path.join(th.GOLDEN, "philox_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((v[:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answer_vectors():
    """The published Philox4x32-10 known-answer vectors (all-zero, all-ones
    and the pi-digits counter and key) are reproduced by the oracle's C
    generator and by the independent Python one."""
    rows = load_philox_kat()
    assert len(rows) == 3
    for ctr, key, want in rows:
        got = oracle.philox4x32_10(np.array(ctr, np.uint32), np.array(key, np.uint32))
        assert list(map(int, got)) == want, (ctr, key, [hex(x) for x in got])
        assert th.philox4x32_10_py(ctr, key) == want


def test_philox_matches_independent_python():
    rng = np.random.default_rng(7)
    for _ in range(300):
        ctr = rng.integers(0, 2 ** 32, 4, dtype=np.uint64)
        key = rng.integers(0, 2 ** 32, 2, dtype=np.uint64)
        got = oracle.philox4x32_10(ctr.astype(np.uint32), key.astype(np.uint32))
        assert list(map(int, got)) == th.philox4x32_10_py(ctr, key)
    # edge counters and keys
    for ctr, key in [([0] * 4, [0, 0]), ([2 ** 32 - 1] * 4, [2 ** 32 - 1] * 2)]:
        got = oracle.philox4x32_10(np.array(ctr, np.uint32), np.array(key, np.uint32))
        assert list(map(int, got)) == th.philox4x32_10_py(ctr, key)


def test_chunks_match_independent_python():
    for seed in (0, 1234, 2 ** 40 + 17):
        for site in (0, 1, 4095, 2 ** 32 - 1):
            for t in (0, 1, 99, 2 ** 32 + 3):
                for stream, n in ((0, 16), (1, 20)):
                    got = oracle.uniform_chunks(seed, site, t, stream, n)
                    assert list(map(int, got)) == th.chunks24_py(seed, site, t, stream, n)


def test_philox_bits_uniform():
    """Chi-square on bytes and per-bit balance over 2^17 output words."""
    words = []
    for s in range(1 << 15):
        words.append(oracle.philox4x32_10(np.array([s, 3, 0, 0], np.uint32),
                                          np.array([1234, 0], np.uint32)))
    w = np.concatenate(words).astype(np.uint64)
    by = np.concatenate([(w >> (8 * b)) & 0xFF for b in range(4)])
    counts = np.bincount(by.astype(np.int64), minlength=256)
    chi2, p = stats.chisquare(counts)
    assert p > 1e-3
    bits = np.array([((w >> b) & 1).mean() for b in range(32)])
    assert np.all(np.abs(bits - 0.5) < 5 * 0.5 / np.sqrt(len(w)))


def test_counter_words_decorrelate():
    """Adjacent sites and steps give uncorrelated normals."""
    z = np.array([oracle.normals(1234, s, 0, 0, 15) for s in range(4000)])
    zt = np.array([oracle.normals(1234, s, 1, 0, 15) for s in range(4000)])
    c = np.corrcoef(np.hstack([z, zt]).T)
    off = c - np.eye(30)
    assert np.abs(off).max() < 5 / np.sqrt(4000)


def test_normals_distribution():
    z = np.concatenate([oracle.normals(99, s, t, 0, 16) for s in range(3000) for t in range(5)])
    n = len(z)
    assert abs(z.mean()) < 5 / np.sqrt(n)
    assert abs(z.var() - 1) < 5 * np.sqrt(2 / n)
    assert abs(stats.kurtosis(z)) < 5 * np.sqrt(24 / n)
    assert stats.kstest(z, "norm").pvalue > 1e-3
    # Box-Muller with 24-bit u1 in (0, 1] bounds |z| by sqrt(48 ln 2)
    assert np.abs(z).max() <= np.sqrt(48 * np.log(2)) + 1e-12


def test_box_muller_mapping_special_values():
    """Consistency of the chunk -> normal map on one pair (not a pin by
    itself; the distribution tests above are the pins)."""
    ch = oracle.uniform_chunks(5, 17, 3, 0, 2)
    u1 = (ch[0] + 1.0) * 2.0 ** -24
    u2 = ch[1] * 2.0 ** -24
    z = oracle.normals(5, 17, 3, 0, 2)
    r = np.sqrt(-2 * np.log(u1))
    assert z[0] == pytest.approx(r * np.cos(2 * np.pi * u2), rel=1e-15, abs=1e-15)
    assert z[1] == pytest.approx(r * np.sin(2 * np.pi * u2), rel=1e-15, abs=1e-15)
