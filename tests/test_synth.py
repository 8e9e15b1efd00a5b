"""Seeded input generators: Philox4x32-10 against its published answers."""
import os

import numpy as np

import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def test_philox_known_answers():
    rows = [l.split() for l in open(GOLD) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = synth.philox4x32_10([v[0]], [v[1]], [v[2]], [v[3]], v[4], v[5])
        assert [int(o[0]) for o in out] == v[6:10]


def test_uniform_points_range_and_determinism():
    X = synth.uniform_points(7, 2, 10000)
    assert X.dtype == np.float32 and X.shape == (2, 10000)
    assert X.min() >= np.float32(-np.pi) and X.max() <= np.float32(np.pi)
    X2 = synth.uniform_points(7, 2, 5000, start=5000)
    assert np.array_equal(X[:, 5000:], X2)
    # uniformity: mean and variance of U[-pi, pi)
    assert abs(X.mean()) < 0.1 and abs(X.var() - np.pi ** 2 / 3) < 0.15


def test_normal_noise_moments():
    z = synth.normal_noise(11, 1, 200000)
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1.0) < 0.01
