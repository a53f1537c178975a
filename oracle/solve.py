"""Linear solves for the oracle (test infrastructure only).

The paper solves every level system to a relative residual of 1e-12
(Sec. 4).  The oracle uses restarted GMRES with modified Gram-Schmidt from
x0 = 0, judged by the true residual |b - D x| / |b|, or a dense LU when the
level is small enough to hold densely.

Parity status: pinned against dense LU solves on small lattices.
"""
from __future__ import annotations

import numpy as np


class NotConverged(RuntimeError):
    pass


def gmres(matvec, b: np.ndarray, tol: float = 1e-12, restart: int = 50,
          maxiter: int = 20000) -> np.ndarray:
    """Restarted GMRES(restart) on a flat complex vector b."""
    bnorm = np.linalg.norm(b)
    x = np.zeros_like(b)
    if bnorm == 0.0:
        return x
    its = 0
    while its < maxiter:
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        if beta <= tol * bnorm:
            return x
        m = restart
        V = np.zeros((m + 1, b.size), dtype=np.complex128)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        V[0] = r / beta
        k_used = 0
        for j in range(m):
            w = matvec(V[j])
            for i in range(j + 1):
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            k_used = j + 1
            its += 1
            if H[j + 1, j] != 0.0:
                V[j + 1] = w / H[j + 1, j]
            # least-squares residual of the small problem
            e1 = np.zeros(j + 2, dtype=np.complex128)
            e1[0] = beta
            y, *_ = np.linalg.lstsq(H[:j + 2, :j + 1], e1, rcond=None)
            res = np.linalg.norm(e1 - H[:j + 2, :j + 1] @ y)
            if res <= 0.5 * tol * bnorm or H[j + 1, j] == 0.0:
                break
        x = x + V[:k_used].T @ y
    r = b - matvec(x)
    if np.linalg.norm(r) > tol * bnorm:
        raise NotConverged("GMRES did not reach %g" % tol)
    return x


class DenseSolver:
    """LU of a dense level matrix, reused across right-hand sides."""

    def __init__(self, A: np.ndarray):
        import scipy.linalg
        self.lu = scipy.linalg.lu_factor(A)
        self._s = scipy.linalg.lu_solve

    def __call__(self, b: np.ndarray) -> np.ndarray:
        return self._s(self.lu, b)


def level_solver(op, tol: float = 1e-12, dense_limit: int = 6144):
    """Returns solve(b) for a level operator: dense LU for n <= dense_limit,
    GMRES otherwise."""
    if op.n <= dense_limit:
        return DenseSolver(op.dense())
    return lambda b: gmres(op.matvec, b, tol=tol)


def relative_residual(matvec, x: np.ndarray, b: np.ndarray) -> float:
    return float(np.linalg.norm(b - matvec(x)) / np.linalg.norm(b))
