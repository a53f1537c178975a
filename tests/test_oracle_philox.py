"""Pins of the oracle's probe generator and of the Z4 variance identity."""
import itertools
import os

import numpy as np
import pytest

from oracle.philox import philox4x32_10, z4_vector, z4_codes, stream_id
from oracle.estimators import offdiag_fro2, mean_var

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(w, 16) for w in line.split()]
        rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("row", _kat())
def test_philox_known_answers(row):
    ctr, key, want = row
    got = philox4x32_10(tuple(np.uint32(c) for c in ctr), tuple(key))
    assert [int(g) for g in got] == want


def test_philox_vectorised_matches_scalar():
    ctr = (np.arange(5, dtype=np.uint32), np.uint32(7), np.uint32(3), np.uint32(9))
    vec = philox4x32_10(ctr, (11, 12))
    for i in range(5):
        sc = philox4x32_10((np.uint32(i), np.uint32(7), np.uint32(3), np.uint32(9)), (11, 12))
        assert all(int(vec[w][i]) == int(sc[w]) for w in range(4))


def test_z4_values_and_frequencies():
    x = z4_vector(200000, seed=101, stream=stream_id(0, 0), probe=3)
    vals = {1, 1j, -1, -1j}
    assert set(np.unique(x).tolist()) <= vals
    codes = z4_codes(200000, 101, 0, 3)
    counts = np.bincount(codes, minlength=4)
    chi2 = np.sum((counts - 50000.0) ** 2 / 50000.0)
    assert chi2 < 16.27  # 3 dof, p = 0.001
    # code -> value map (1, i, -1, -i)
    np.testing.assert_array_equal(x, np.array([1, 1j, -1, -1j])[codes])


def test_z4_streams_and_probes_differ_and_are_uncorrelated():
    a = z4_vector(50000, 5, stream_id(0, 1), 0)
    b = z4_vector(50000, 5, stream_id(0, 2), 0)
    c = z4_vector(50000, 5, stream_id(0, 1), 1)
    d = z4_vector(50000, 6, stream_id(0, 1), 0)
    for u in (b, c, d):
        assert abs(np.vdot(a, u)) / 50000 < 5 / np.sqrt(50000)
    np.testing.assert_array_equal(a, z4_vector(50000, 5, stream_id(0, 1), 0))


def test_z4_counter_uses_64bit_index():
    """Entry i and entry i + 2^32 use different counters (high word)."""
    from oracle.philox import z4_codes_at
    k = np.arange(256, dtype=np.uint64)
    lo = z4_codes_at(k, 1, 0, 0)
    hi = z4_codes_at(k + np.uint64(1 << 32), 1, 0, 0)
    assert np.mean(lo == hi) < 0.5


def test_z4_variance_identity_brute_force():
    """Exact mean and variance of x^H A x over all 4^n Z4 vectors equal tr(A)
    and ||offdiag(A)||_F^2 (Sec. 1, eq. variance-Frobenius-Relation)."""
    rng = np.random.default_rng(0)
    n = 5
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    z4 = np.array([1, -1, 1j, -1j])
    vals = []
    for c in itertools.product(range(4), repeat=n):
        x = z4[list(c)]
        vals.append(np.vdot(x, A @ x))
    vals = np.array(vals)
    assert abs(vals.mean() - np.trace(A)) < 1e-12
    var = np.mean(np.abs(vals - np.trace(A)) ** 2)
    assert abs(var - offdiag_fro2(A)) < 1e-10 * offdiag_fro2(A)


def test_variance_estimator_is_unbiased_form():
    X = np.array([1 + 1j, 2 - 1j, -1 + 0.5j])
    mu, v = mean_var(X)
    assert abs(mu - X.mean()) < 1e-15
    assert abs(v - np.sum(np.abs(X - X.mean()) ** 2) / 2) < 1e-15
