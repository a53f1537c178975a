"""Inexact deflation of the Hutchinson estimator (oracle; test infrastructure).

What the paper fixes (Sec. 2.1, "Deflation" and "Deflation for the Dirac
operator"; setup in Sec. 4.2):

* tr(A) = tr((I - Pi) A) + tr(Pi A) for an orthogonal projector Pi = V V^H
  (eq. deflation-general); with A = D^-1, tr(Pi A) = tr(V^H D^-1 V) is
  computed exactly from k solves with the columns of V.
* The deflated estimator with N probes x^n (eq. deflated-estimator):
  (1/N) sum_n (x^n)^H (I - V V^H) D^-1 x^n + tr(V^H D^-1 V).
* V holds approximate eigenvectors of the Hermitian Q = Gamma5 D belonging to
  its eigenvalues of smallest modulus (right singular vectors of D for its
  smallest singular values, so the projector removes the largest singular
  values of D^-1); in the experiments five iterations of an inverse block
  power method on Gamma5 D, every inner inversion to a relative residual of
  1e-6, with k = 128.

Readings (the paper leaves these open; also listed in the design notes):

* Start block: k Z4 vectors (Sec. 1, eq. z4) from the counter generator on
  stream 256*0 + 9 (kind 9: deflation basis), probe index = column index.
* Orthonormalisation after the start and after every power step: modified
  Gram-Schmidt with one re-orthogonalisation pass over the columns in order,
  positive real diag(R) (the same QR as the multigrid setup: the result is
  the unique Q of the QR factorisation, so any QR algorithm gives it up to
  rounding).
* Power step: W = Q^-1 V = D^-1 Gamma5 V, one solve per column, then V = QR(W).
  No Rayleigh-Ritz step: the projector depends only on the span of V.
* Probes of the stochastic term: Z4 on stream 256*0 + 10 (kind 10).

Parity status: pinned by a diagonal Q worked out by hand (inverse power
iterations), convergence of the span to the k smallest |eigenvalues| of the
dense Q, the trace split tr((I-Pi)D^-1) + tr(V^H D^-1 V) = tr(D^-1), the
optimal Frobenius reduction of eq. Frobenius-reduction-singular, and the Z4
variance identity (tests/test_oracle_deflation.py).
"""
from __future__ import annotations

import numpy as np

from .philox import z4_vector, stream_id

KIND_DEFL_BASIS = 9
KIND_DEFL_PROBE = 10


def mgs2(W: np.ndarray) -> np.ndarray:
    """Orthonormal columns of W (n x k) by modified Gram-Schmidt with one
    re-orthogonalisation pass, columns in order, positive real diag(R)."""
    n, k = W.shape
    Q = np.zeros_like(W)
    for j in range(k):
        w = W[:, j].copy()
        n0 = np.linalg.norm(w)
        for _ in range(2):
            for i in range(j):
                w = w - np.vdot(Q[:, i], w) * Q[:, i]
        nrm = np.linalg.norm(w)
        if n0 == 0.0 or nrm < 1e-12 * n0:
            raise np.linalg.LinAlgError("deflation block lost rank at column %d" % j)
        Q[:, j] = w / nrm
    return Q


def gamma5_fine(v: np.ndarray) -> np.ndarray:
    """Gamma5 on a fine vector (dof = 3*spin + colour, gamma5 = diag(1,1,-1,-1))."""
    s = v.reshape(v.shape[:-1] + (-1, 12)).copy()
    s[..., 6:] *= -1.0
    return s.reshape(v.shape)


def start_block(n: int, k: int, seed: int) -> np.ndarray:
    """k Z4 columns on the deflation-basis stream (kind 9, level 0)."""
    return np.stack([z4_vector(n, seed, stream_id(0, KIND_DEFL_BASIS), j) for j in range(k)], axis=1)


def inverse_block_power(solve_q, V0: np.ndarray, iters: int) -> np.ndarray:
    """V = QR(V0), then `iters` times V = QR(Q^-1 V); solve_q(b) returns Q^-1 b."""
    V = mgs2(V0)
    for _ in range(iters):
        W = np.stack([solve_q(V[:, j]) for j in range(V.shape[1])], axis=1)
        V = mgs2(W)
    return V


def deflation_basis(solve_d, n: int, k: int, seed: int, iters: int = 5) -> np.ndarray:
    """The inexact deflation basis of the Dirac operator: inverse block power
    on Q = Gamma5 D, with Q^-1 b = D^-1 (Gamma5 b); solve_d(b) returns D^-1 b
    (to whatever tolerance the caller's solver uses)."""
    return inverse_block_power(lambda b: solve_d(gamma5_fine(b)), start_block(n, k, seed), iters)


def deflated_exact_term(solve_d, V: np.ndarray) -> complex:
    """tr(V^H D^-1 V) = sum_j v_j^H D^-1 v_j (k solves)."""
    return complex(sum(np.vdot(V[:, j], solve_d(V[:, j])) for j in range(V.shape[1])))


def deflated_samples(solve_d, V: np.ndarray, seed: int, nprobe: int, first: int = 0) -> np.ndarray:
    """Per-probe X = x^H (I - V V^H) D^-1 x for Z4 probes on kind 10."""
    n = V.shape[0]
    out = np.zeros(nprobe, dtype=np.complex128)
    for p in range(nprobe):
        x = z4_vector(n, seed, stream_id(0, KIND_DEFL_PROBE), first + p)
        px = x - V @ (V.conj().T @ x)
        out[p] = np.vdot(px, solve_d(x))
    return out
