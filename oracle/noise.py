"""Probe distributions other than Z4, and probing (coloured) sources for
loops (oracle; test infrastructure only).

What the paper fixes (Sec. 1, after eq. variance-Frobenius-Relation):
Hutchinson's estimator needs i.i.d. entries with E[x_i] = 0 and
E[conj(x_i) x_j] = delta_ij.  Besides Z4 it names the uniform distribution on
the unit circle (same variance as Z4), Z2 = {-1, 1}, and the standard normal
distribution N(0, 1).  For the loops it names probing and related structured
noise, combined with the multilevel decomposition, as the next step (Sec. 5).

Readings (the paper leaves these open; also listed in the design notes):

* Every distribution is drawn from the same Philox4x32-10 words as Z4
  (philox.py): w = philox(counter = (i lo, i hi, probe, stream), key = seed).
    Z4:    (1, i, -1, -i)[w0 >> 30]                         (philox.py)
    Z2:    1 - 2 (w0 >> 31)
    U(1):  exp(2 pi i (w0 + 1/2) 2^-32)
    N(0,1) (real): Box and Muller (1958) on u1 = (w0 + 1) 2^-32 in (0, 1],
           u2 = w1 2^-32: sqrt(-2 ln u1) cos(2 pi u2)
* The variance of the real Gaussian estimator is (1/2N) ||A + A^T||_F^2 (a
  direct computation of the fourth moments); the paper prints (1/N) for
  it, which is the value for E[x_i^2] = 2.  The tests pin the factor 1/2.
* Probing: sites are coloured by a p^4 block pattern,
  colour(x) = (x mod p) + p((y mod p) + p((z mod p) + p(t mod p))),
  so two sites of one colour are at least p apart along some axis; a probe is
  the sum over colours c of eta_c^H A eta_c with eta_c the noise restricted
  to the sites of colour c (one solve per colour).  This keeps E = tr(A) and
  removes from the variance every off-diagonal entry A_ij between sites of
  different colours: Var = sum_{i != j, colour(i) = colour(j)} |A_ij|^2 for
  Z4 noise.  p = 1 is plain (one colour).

Parity status: pinned by brute force over all Z2 / Z4 vectors on small
matrices (exact variances), moment and Kolmogorov-Smirnov tests of the
generated distributions, a Monte Carlo pin of the Gaussian variance and the
coloured Z4 variance identity (tests/test_oracle_noise.py).
"""
from __future__ import annotations

import numpy as np

from .philox import philox4x32_10, MASK32

NOISE_Z4, NOISE_Z2, NOISE_U1, NOISE_GAUSS = 0, 1, 2, 3
NOISE_NAMES = {"z4": NOISE_Z4, "z2": NOISE_Z2, "u1": NOISE_U1, "gauss": NOISE_GAUSS}

_Z4 = np.array([1.0, 1.0j, -1.0, -1.0j], dtype=np.complex128)


def _words(n: int, seed: int, stream: int, probe: int):
    i = np.arange(n, dtype=np.uint64)
    ctr = ((i & MASK32).astype(np.uint32), (i >> np.uint64(32)).astype(np.uint32),
           np.uint32(probe), np.uint32(stream))
    key = (int(seed) & 0xFFFFFFFF, (int(seed) >> 32) & 0xFFFFFFFF)
    return philox4x32_10(ctr, key)


def noise_vector(n: int, seed: int, stream: int, probe: int, kind: int = NOISE_Z4) -> np.ndarray:
    """Probe vector of n entries for (seed, stream, probe) from distribution kind."""
    w0, w1, _, _ = _words(n, seed, stream, probe)
    if kind == NOISE_Z4:
        return _Z4[(w0 >> np.uint32(30)).astype(np.int64)]
    if kind == NOISE_Z2:
        return (1.0 - 2.0 * (w0 >> np.uint32(31)).astype(np.float64)).astype(np.complex128)
    if kind == NOISE_U1:
        theta = 2.0 * np.pi * (w0.astype(np.float64) + 0.5) * 2.0 ** -32
        return np.exp(1j * theta)
    if kind == NOISE_GAUSS:
        u1 = (w0.astype(np.float64) + 1.0) * 2.0 ** -32
        u2 = w1.astype(np.float64) * 2.0 ** -32
        return (np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)).astype(np.complex128)
    raise ValueError("unknown noise kind %r" % kind)


def site_colours(dims, p: int) -> np.ndarray:
    """Colour of every site (lexicographic s = x + X(y + Y(z + Z t))) for the
    p^4 block pattern; p must divide every extent."""
    X, Y, Z, T = dims
    for L in dims:
        if L % p != 0:
            raise ValueError("probing distance %d does not divide the lattice %s" % (p, dims))
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    c = (x % p) + p * ((y % p) + p * ((z % p) + p * (t % p)))
    return c.reshape(-1)


def colour_masks(dims, p: int, dof: int = 12):
    """Boolean masks over the dof of a level vector, one per colour."""
    col = np.repeat(site_colours(dims, p), dof)
    return [col == c for c in range(p ** 4)]
