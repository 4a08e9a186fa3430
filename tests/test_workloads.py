"""Seeded input generators: reproducibility and the stated distributions."""
import numpy as np

import workloads as W


def test_seeded_and_reproducible():
    a = W.Cfg2(N=64).coef()
    b = W.Cfg2(N=64).coef()
    assert np.array_equal(a, b)
    assert not np.array_equal(W.normal_block(1, 4, 4), W.normal_block(2, 4, 4))
    assert W.seed_for(3, W.S0, 7) == 3071


def test_grf_covariance():
    # pooled over seeds: unit variance, correlation exp(-d^2/(2 l^2)) at lag d
    N, l = 128, 0.1
    fields = [W.grf_field(s, N, l, 1.0) for s in range(40)]
    g = np.stack(fields)
    assert abs(g.var() - 1.0) < 0.1
    for lag in (6, 13):
        d = lag / N
        corr = np.mean(g[:, :, :-lag] * g[:, :, lag:]) / g.var()
        assert abs(corr - np.exp(-d * d / (2 * l * l))) < 0.08


def test_checkerboard_and_aniso():
    a = W.checkerboard_3d(5, 32, 4)
    assert a.shape == (32, 32, 32) and set(np.unique(a)) <= {1.0, 1e3}
    assert np.all(a[:8, :8, :8] == a[0, 0, 0])
    s = W.checkerboard_3d(0, 16, 2, strict=True)
    assert s[0, 0, 0] == 1.0 and s[0, 0, 8] == 1e3
    side, eps, th = W.aniso_batch(0, 500)
    assert set(np.unique(side)) == set(W.ANISO_SIDES)
    assert eps.min() >= 1e-3 and eps.max() <= 1.0 and th.min() >= 0 and th.max() <= np.pi
