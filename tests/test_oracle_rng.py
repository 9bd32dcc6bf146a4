"""Oracle RNG pins: Philox4x32-10 known-answer vectors and an independent
pure-Python implementation of the published round function."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        rows.append([int(x, 16) for x in line.split()])
    return rows


def py_philox(ctr, key):
    """Philox4x32-10 as published: 10 rounds, multipliers 0xD2511F53/0xCD9E8D57,
    Weyl key bumps 0x9E3779B9/0xBB67AE85."""
    c = list(ctr)
    k0, k1 = key
    for _ in range(10):
        p0 = 0xD2511F53 * c[0]
        p1 = 0xCD9E8D57 * c[2]
        c = [((p1 >> 32) ^ c[1] ^ k0) & 0xFFFFFFFF, p1 & 0xFFFFFFFF,
             ((p0 >> 32) ^ c[3] ^ k1) & 0xFFFFFFFF, p0 & 0xFFFFFFFF]
        k0 = (k0 + 0x9E3779B9) & 0xFFFFFFFF
        k1 = (k1 + 0xBB67AE85) & 0xFFFFFFFF
    return c


def test_known_answer_vectors(oracle_lib):
    for row in _kat():
        out = oracle_lib.philox(row[:4], row[4:6])
        assert [int(x) for x in out] == row[6:10]
        assert py_philox(row[:4], row[4:6]) == row[6:10]


def test_matches_python_reference(oracle_lib):
    rng = np.random.default_rng(3)
    for _ in range(200):
        ctr = [int(x) for x in rng.integers(0, 2 ** 32, 4)]
        key = [int(x) for x in rng.integers(0, 2 ** 32, 2)]
        assert [int(x) for x in oracle_lib.philox(ctr, key)] == py_philox(ctr, key)


def test_uniform_chi2(oracle_lib):
    # 24-bit uniforms from consecutive counters: chi-square over 16 bins
    vals = []
    for i in range(4000):
        vals += [int(x) >> 8 for x in oracle_lib.philox([i, 7, 0, 0], [1, 2])]
    u = np.array(vals) / 2.0 ** 24
    h, _ = np.histogram(u, bins=16, range=(0, 1))
    e = len(u) / 16
    chi2 = ((h - e) ** 2 / e).sum()
    assert chi2 < 40.0  # 15 dof: p ~ 5e-4
