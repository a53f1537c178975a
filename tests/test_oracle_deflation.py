"""Pins of the oracle's inexact deflation (Sec. 2.1, eq. deflated-estimator;
setup of Sec. 4.2): a hand-worked diagonal case of the inverse block power
method, convergence to the small-|eigenvalue| space of the dense Gamma5 D,
the exact trace split, the optimal Frobenius reduction, unbiasedness and the
Z4 variance identity."""
import numpy as np
import pytest

from lattice_inputs import gauge_field
from oracle.dirac import WilsonClover
from oracle.philox import z4_vector, stream_id
from oracle import deflation as DF
from oracle import estimators as E


def test_inverse_power_on_a_diagonal_matrix_by_hand():
    """Q = diag(1, 2, 4, 8), start (1, 1, 1, 1): QR gives (1,1,1,1)/2, one
    inverse power step gives (8, 4, 2, 1)/sqrt(85), two give
    (64, 16, 4, 1)/sqrt(4369)."""
    q = np.array([1.0, 2.0, 4.0, 8.0])
    V0 = np.ones((4, 1), dtype=complex)
    np.testing.assert_allclose(DF.inverse_block_power(lambda b: b / q, V0, 0)[:, 0], 0.5, atol=1e-15)
    v1 = DF.inverse_block_power(lambda b: b / q, V0, 1)[:, 0]
    np.testing.assert_allclose(v1, np.array([8, 4, 2, 1]) / np.sqrt(85.0), atol=1e-15)
    v2 = DF.inverse_block_power(lambda b: b / q, V0, 2)[:, 0]
    np.testing.assert_allclose(v2, np.array([64, 16, 4, 1]) / np.sqrt(4369.0), atol=1e-15)
    # a block of two converges to span(e1, e2), the two smallest |eigenvalues|
    # (also with a negative eigenvalue of larger modulus present)
    q2 = np.array([1.0, -2.0, 4.0, -8.0])
    V0 = np.array([[1, 1], [1, -1], [1, 1], [1, -1]], dtype=complex)
    V = DF.inverse_block_power(lambda b: b / q2, V0, 80)
    np.testing.assert_allclose(V.conj().T @ V, np.eye(2), atol=1e-14)
    for e in (0, 1):
        x = np.zeros(4)
        x[e] = 1
        assert np.linalg.norm(x - V @ (V.conj().T @ x)) < 1e-12


def test_mgs2_positive_diagonal_matches_numpy_qr():
    rng = np.random.default_rng(1)
    W = rng.standard_normal((40, 6)) + 1j * rng.standard_normal((40, 6))
    Q = DF.mgs2(W)
    Qn, R = np.linalg.qr(W)
    ph = np.diag(R) / np.abs(np.diag(R))
    np.testing.assert_allclose(Q, Qn * ph[None, :], atol=1e-13)
    with pytest.raises(np.linalg.LinAlgError):
        DF.mgs2(np.stack([W[:, 0], 2 * W[:, 0]], axis=1))


@pytest.fixture(scope="module")
def dense():
    U = gauge_field((4, 4, 4, 4), 0.5, 12)
    D = WilsonClover(U, 0.05, 1.0)
    A = D.dense()
    Dinv = np.linalg.inv(A)
    return D, A, Dinv


def test_gamma5_d_is_hermitian(dense):
    D, A, _ = dense
    n = A.shape[0]
    G5A = np.stack([DF.gamma5_fine(A[:, j]) for j in range(n)], axis=1)
    assert np.abs(G5A - G5A.conj().T).max() < 1e-12 * np.abs(G5A).max()


def test_basis_converges_to_smallest_modes_and_optimal_frobenius():
    """A Gamma5-hermitian D = Gamma5 Q with Q = W diag(lam) W^H of a known
    spectrum (four sites, n = 48; |lam| from 0.5 to 24 with a gap of two
    between the fourth and fifth smallest): with exact solves the span of the
    k = 4 basis converges to the eigenvectors of the four smallest |lam|, and
    ||(I - Pi) D^-1||_F^2 reaches ||D^-1||_F^2 - sum_{i<=k} 1/lam_i^2, the
    least a rank-k projection can leave (eq. Frobenius-reduction-singular)."""
    rng = np.random.default_rng(3)
    n, k = 48, 4
    W, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    mags = np.concatenate([[0.5, 0.6, 0.7, 0.8], np.linspace(1.6, 24.0, n - 4)])
    lam = mags * np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    Q = W @ np.diag(lam) @ W.conj().T
    Dm = np.stack([DF.gamma5_fine(Q[:, j]) for j in range(n)], axis=1)  # D = Gamma5 Q
    Dinv = np.linalg.inv(Dm)

    def solve(b):
        return Dinv @ b

    f_opt = np.sum(1.0 / lam ** 2) - np.sum(1.0 / lam[:k] ** 2)
    V = DF.deflation_basis(solve, n, k, seed=5, iters=60)
    f = np.linalg.norm(Dinv - V @ (V.conj().T @ Dinv)) ** 2
    assert abs(f - f_opt) < 1e-10 * f_opt
    Wk = W[:, :k]
    assert np.linalg.norm(Wk - V @ (V.conj().T @ Wk)) < 1e-10
    # fewer iterations leave more: the Frobenius norm falls towards the optimum
    fs = []
    for it in (0, 1, 5):
        Vi = DF.deflation_basis(solve, n, k, seed=5, iters=it)
        fs.append(np.linalg.norm(Dinv - Vi @ (Vi.conj().T @ Dinv)) ** 2)
    assert fs[0] > fs[1] > fs[2] >= f_opt * (1 - 1e-12)
    # the start block is the Z4 draw of kind 9, orthonormalised
    x0 = z4_vector(n, 5, stream_id(0, DF.KIND_DEFL_BASIS), 0)
    V0 = DF.deflation_basis(solve, n, k, seed=5, iters=0)
    np.testing.assert_allclose(V0[:, 0], x0 / np.linalg.norm(x0), atol=1e-15)


def test_trace_split_samples_and_variance(dense):
    D, A, Dinv = dense
    n, k = A.shape[0], 8

    def solve(b):
        return Dinv @ b

    V = DF.deflation_basis(solve, n, k, seed=7, iters=5)
    V0 = DF.deflation_basis(solve, n, k, seed=7, iters=0)
    Pi = V @ V.conj().T
    Adef = (np.eye(n) - Pi) @ Dinv
    exact = DF.deflated_exact_term(solve, V)
    # eq. deflation-general: tr((I - Pi) A) + tr(V^H A V) = tr(A)
    assert abs(np.trace(Adef) + exact - np.trace(Dinv)) < 1e-12 * abs(np.trace(Dinv))
    N = 64
    X = DF.deflated_samples(solve, V, seed=9, nprobe=N)
    for p in range(3):
        x = z4_vector(n, 9, stream_id(0, DF.KIND_DEFL_PROBE), p)
        assert abs(X[p] - np.vdot(x, Adef @ x)) < 1e-12 * abs(X[p])
    sig2 = E.offdiag_fro2(Adef)
    assert abs(X.mean() - np.trace(Adef)) < 5 * np.sqrt(sig2 / N)
    _, v = E.mean_var(X)
    assert 0.4 < v / sig2 < 2.0
    # deflation lowers the Frobenius norm and the Z4 variance below plain
    # Hutchinson's, and the power steps lower the norm below the random start's
    assert sig2 < E.offdiag_fro2(Dinv)
    f5 = np.linalg.norm(Adef) ** 2
    f0 = np.linalg.norm(Dinv - V0 @ (V0.conj().T @ Dinv)) ** 2
    assert f5 < f0 < np.linalg.norm(Dinv) ** 2
