"""Pins of the oracle's probe distributions and probing sources (Sec. 1 after
eq. variance-Frobenius-Relation; Sec. 5 for probing): generated values and
moments, exact variances by brute force over every Z2 / Z4 vector, the
Gaussian variance by Monte Carlo, and the coloured Z4 variance identity."""
import itertools

import numpy as np
import pytest
import scipy.stats

from oracle.noise import (noise_vector, site_colours, colour_masks, NOISE_Z4, NOISE_Z2, NOISE_U1,
                          NOISE_GAUSS)
from oracle.philox import z4_vector


def _rand_matrix(n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))


def test_z4_kind_equals_the_z4_generator():
    assert np.array_equal(noise_vector(1000, 7, 3, 5, NOISE_Z4), z4_vector(1000, 7, 3, 5))


def test_distributions_values_and_moments():
    n = 200000
    z2 = noise_vector(n, 11, 0, 0, NOISE_Z2)
    assert set(np.unique(z2.real)) == {-1.0, 1.0} and np.all(z2.imag == 0)
    assert abs(z2.real.mean()) < 5 / np.sqrt(n)
    u1 = noise_vector(n, 11, 0, 0, NOISE_U1)
    np.testing.assert_allclose(np.abs(u1), 1.0, atol=1e-15)
    assert abs(u1.mean()) < 5 / np.sqrt(n) and abs((u1 ** 2).mean()) < 5 / np.sqrt(n)
    theta = np.mod(np.angle(u1), 2 * np.pi) / (2 * np.pi)
    assert scipy.stats.kstest(theta, "uniform").pvalue > 1e-3
    g = noise_vector(n, 11, 0, 0, NOISE_GAUSS)
    assert np.all(g.imag == 0)
    x = g.real
    assert abs(x.mean()) < 5 / np.sqrt(n)
    assert abs((x ** 2).mean() - 1) < 5 * np.sqrt(2 / n)
    assert abs((x ** 4).mean() - 3) < 5 * np.sqrt(96 / n)
    assert scipy.stats.kstest(x, "norm").pvalue > 1e-3
    # the same words feed the distributions: Z2 is the sign of the Z4 code's top bit
    z4 = noise_vector(n, 11, 0, 0, NOISE_Z4)
    assert np.array_equal(z2.real > 0, (z4 == 1) | (z4 == 1j))


def _brute_variance(A, values):
    n = A.shape[0]
    X = []
    for v in itertools.product(values, repeat=n):
        x = np.array(v)
        X.append(np.vdot(x, A @ x))
    X = np.array(X)
    return X.mean(), np.mean(np.abs(X - X.mean()) ** 2)


def test_exact_variances_by_brute_force():
    """All 2^n (Z2) and 4^n (Z4) vectors of a random 6 x 6 complex matrix:
    both unbiased; Var = ||offdiag A||_F^2 for Z4 and
    (1/2)||offdiag(A + A^T)||_F^2 for Z2 (Sec. 1)."""
    A = _rand_matrix(6, 3)
    off = A - np.diag(np.diag(A))
    m4, v4 = _brute_variance(A, [1, 1j, -1, -1j])
    assert abs(m4 - np.trace(A)) < 1e-12 and abs(v4 - np.sum(np.abs(off) ** 2)) < 1e-10
    m2, v2 = _brute_variance(A, [1, -1])
    S = A + A.T
    assert abs(m2 - np.trace(A)) < 1e-12
    assert abs(v2 - 0.5 * np.sum(np.abs(S - np.diag(np.diag(S))) ** 2)) < 1e-10


def test_gaussian_and_u1_variances_by_monte_carlo():
    """Real N(0,1) entries: Var = (1/2)||A + A^T||_F^2 (the factor 1/2 is
    a reading: the printed (1/N)||A + A^T||_F^2 is twice this); U(1): the Z4
    variance ||offdiag A||_F^2.  Checked with 40000 probes of a 4 x 4 matrix."""
    A = _rand_matrix(4, 5)
    N = 40000
    Xg = np.array([np.vdot(x, A @ x) for x in (noise_vector(4, 21, 0, p, NOISE_GAUSS) for p in range(N))])
    want_g = 0.5 * np.sum(np.abs(A + A.T) ** 2)
    vg = np.mean(np.abs(Xg - Xg.mean()) ** 2)
    assert abs(Xg.mean() - np.trace(A)) < 5 * np.sqrt(want_g / N)
    assert abs(vg / want_g - 1) < 0.06
    Xu = np.array([np.vdot(x, A @ x) for x in (noise_vector(4, 22, 0, p, NOISE_U1) for p in range(N))])
    want_u = np.sum(np.abs(A - np.diag(np.diag(A))) ** 2)
    vu = np.mean(np.abs(Xu - Xu.mean()) ** 2)
    assert abs(vu / want_u - 1) < 0.06


def test_site_colours_by_hand():
    dims = (4, 2, 2, 2)
    c = site_colours(dims, 2)
    # site (x, y, z, t) = (3, 1, 0, 1): colour 1 + 2*(1 + 2*(0 + 2*1)) = 11
    s = 3 + 4 * (1 + 2 * (0 + 2 * 1))
    assert c[s] == 11
    assert sorted(np.unique(c)) == list(range(16))
    # one colour per site, equal counts; p = 1 is a single colour
    assert np.all(np.bincount(c) == 32 // 16)
    assert np.all(site_colours(dims, 1) == 0)
    with pytest.raises(ValueError):
        site_colours((6, 2, 2, 2), 4)


def test_coloured_z4_variance_identity():
    """sum_c eta_c^H A eta_c over the colours of a 2^4 pattern on a 2^4 lattice
    with one dof per site (16 sites, one per colour): unbiased with variance
    sum over i != j of equal colour |A_ij|^2 = 0 here (every colour holds one
    site); with two dof per site, the same-site off-diagonal entries remain."""
    dims = (2, 2, 2, 2)
    n = 16
    A = _rand_matrix(n, 9)
    masks = colour_masks(dims, 2, dof=1)
    vals = []
    for p in range(200):
        eta = noise_vector(n, 4, 0, p, NOISE_Z4)
        vals.append(sum(np.vdot(np.where(m, eta, 0), A @ np.where(m, eta, 0)) for m in masks))
    np.testing.assert_allclose(vals, np.trace(A), atol=1e-12)
    # two dof per site: Var = sum_s (|A[s0, s1]|^2 + |A[s1, s0]|^2)
    n2 = 32
    A2 = _rand_matrix(n2, 10)
    masks2 = colour_masks(dims, 2, dof=2)
    X = []
    for p in range(4000):
        eta = noise_vector(n2, 6, 0, p, NOISE_Z4)
        X.append(sum(np.vdot(np.where(m, eta, 0), A2 @ np.where(m, eta, 0)) for m in masks2))
    X = np.array(X)
    want = sum(abs(A2[2 * s, 2 * s + 1]) ** 2 + abs(A2[2 * s + 1, 2 * s]) ** 2 for s in range(16))
    assert abs(X.mean() - np.trace(A2)) < 5 * np.sqrt(want / len(X))
    assert abs(np.mean(np.abs(X - X.mean()) ** 2) / want - 1) < 0.1
