"""Seeded synthetic inputs shared by the CPU oracle and the GPU library.

This module holds no arithmetic of the trace-estimation method: it only
draws gauge fields and random test vectors.  Both sides receive these arrays
as inputs; neither side's results feed back into this module.

Layouts (all complex128, C order):
  gauge field : [T][Z][Y][X][mu=0..3 (x,y,z,t)][3][3]  -- U_mu(x)_{ab}
  spinor      : [..., T][Z][Y][X][4 spin][3 colour]
so that the flattened site index is s = x + X*(y + Y*(z + Z*t)).

Gauge recipe (stand-in for the paper's RQCD/CLS ensembles, which are not
available): every link is U = exp(i*eps*H) with H = sum_a w_a lambda_a / 2,
w_a ~ N(0,1) i.i.d. per link (lambda_a: Gell-Mann matrices), computed exactly
through the eigendecomposition of H and then re-unitarised to SU(3) (rows 1-2
by Gram-Schmidt, row 3 = conj(row1 x row2)).  "Link roughness" is eps.
"""
from __future__ import annotations

import numpy as np

__all__ = ["gell_mann", "gauge_field", "unit_gauge", "random_spinor",
           "random_su3", "site_volume"]


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices, shape (8, 3, 3)."""
    l = np.zeros((8, 3, 3), dtype=np.complex128)
    l[0, 0, 1] = l[0, 1, 0] = 1
    l[1, 0, 1] = -1j; l[1, 1, 0] = 1j
    l[2, 0, 0] = 1; l[2, 1, 1] = -1
    l[3, 0, 2] = l[3, 2, 0] = 1
    l[4, 0, 2] = -1j; l[4, 2, 0] = 1j
    l[5, 1, 2] = l[5, 2, 1] = 1
    l[6, 1, 2] = -1j; l[6, 2, 1] = 1j
    l[7, 0, 0] = l[7, 1, 1] = 1 / np.sqrt(3); l[7, 2, 2] = -2 / np.sqrt(3)
    return l


def site_volume(dims) -> int:
    X, Y, Z, T = dims
    return int(X) * int(Y) * int(Z) * int(T)


def _reunitarise(U: np.ndarray) -> np.ndarray:
    r0 = U[..., 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = U[..., 1, :]
    r1 = r1 - np.sum(r0.conj() * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.conj(np.cross(r0, r1))
    return np.stack([r0, r1, r2], axis=-2)


def random_su3(shape, eps: float, rng: np.random.Generator) -> np.ndarray:
    """SU(3) matrices exp(i*eps*H) of the recipe above, shape (*shape, 3, 3)."""
    shape = tuple(shape)
    n = int(np.prod(shape)) if shape else 1
    out = np.empty((n, 3, 3), dtype=np.complex128)
    lam = gell_mann() / 2.0
    chunk = 1 << 20
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        w = rng.standard_normal((hi - lo, 8))
        H = np.einsum("na,aij->nij", w, lam)
        ev, vec = np.linalg.eigh(H)
        out[lo:hi] = np.einsum("nab,nb,ncb->nac", vec, np.exp(1j * eps * ev),
                               vec.conj())
    out = _reunitarise(out)
    return out.reshape(shape + (3, 3))


def gauge_field(dims, eps: float, seed: int) -> np.ndarray:
    """Seeded rough SU(3) gauge field, shape (T, Z, Y, X, 4, 3, 3)."""
    X, Y, Z, T = (int(d) for d in dims)
    rng = np.random.default_rng(seed)
    return random_su3((T, Z, Y, X, 4), eps, rng)


def unit_gauge(dims) -> np.ndarray:
    X, Y, Z, T = (int(d) for d in dims)
    U = np.zeros((T, Z, Y, X, 4, 3, 3), dtype=np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1.0
    return U


def random_spinor(dims, seed: int, batch: int | None = None) -> np.ndarray:
    """Complex Gaussian spinor field(s), shape ([batch,] T, Z, Y, X, 4, 3)."""
    X, Y, Z, T = (int(d) for d in dims)
    rng = np.random.default_rng(seed)
    shape = ((batch,) if batch is not None else ()) + (T, Z, Y, X, 4, 3)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
