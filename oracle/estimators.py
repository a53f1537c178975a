"""Hutchinson per-probe values for every decomposition (oracle; test infra).

Each per-probe value X is computed by its definition: draw the Z4 probe,
apply the operator through solves and transfers, take the inner product.

tr(D^-1), Hutchinson (Sec. 1, eq. Hutchinson): X = x^H D^-1 x.
Oblique MG-MLMC (Sec. 2.2, eqs. Al_def and oblique-deflation):
  M_l = D_l^-1 - P_l D_{l+1}^-1 P_l^H, X = x^H D_l^-1 x - (P_l^H x)^H D_{l+1}^-1 P_l^H x.
Orthogonal MG-MLMC (Sec. 3, eqs. OandF_def and the decomposition after it):
  O_l = (I - P_l P_l^H) D_l^-1 (I - P_l P_l^H): y = (I - P P^H) x, X = y^H D_l^-1 y;
  F_l = P_l^H D_l^-1 P_l - D_{l+1}^-1 (x on level l+1):
        X = (P_l x)^H D_l^-1 P_l x - x^H D_{l+1}^-1 x;
  coarsest: X = x^H D_L^-1 x.
Probe streams: stream = 256*level + kind (see philox.py).

Connected correlator (Sec. 1.1 eq. connected-G, Sec. 4.1 eqs. G-ij, G-split):
with B~ := Gamma5 B^H Gamma5,
  tr(B_r(t1,t') G5 B_s(t',t1) G5) = tr(B_r(t1,t') B~_s(t1,t')^H),
which the time-diluted Z4 source eta_{t'} (eta restricted to slice t')
estimates as sum_{x in t1} (B~_s eta_{t'})(x)^H (B_r eta_{t'})(x), t1 = t+t'.
Orthogonal terms (accumulated transfers read as P_hat_{l-1}, 0-based below):
  J_l = (I - Pi_l) D_l^-1,             J~_l = D_l^-1 (I - Pi_l)
  K_l = Pi_l D_l^-1 - P_l D_{l+1}^-1 P_l^H,   K~_l = D_l^-1 Pi_l - P_l D_{l+1}^-1 P_l^H
  coarsest D_L^-1 (Gamma5-hermitian, B~ = B); all embedded with P_hat.
Oblique terms: B_l = P_hat (D_l^-1 - P_l D_{l+1}^-1 P_l^H) P_hat^H, B~ = B.
A term's probe count is that of the finest level it touches (Sec. 4.1).

Disconnected loops (Sec. 4.3 eq. trace_equality_disconnected): for a full
volume Z4 eta, X(t, Gamma) = sum_{x in t} eta(x)^H Gamma (B eta)(x).

Probe entries are Z4 by default; every sample function also takes the other
distributions of noise.py (Z2, U(1), real Gaussian), and the loops take
probing (coloured) sources.

Variance estimator (Sec. 4): V = sum |X_i - mean|^2 / (N - 1).
MLMC sample sizes (Sec. 2.2 eq. MLMC-Nl):
  N_l = eps^-2 sqrt(V_l / C_l) sum_i sqrt(V_i C_i).

Parity status: pinned by dense exact traces, telescoping identities and the
Z4 variance identity on small lattices (tests/test_oracle_estimators.py).
"""
from __future__ import annotations

import numpy as np

from .philox import (stream_id, KIND_PLAIN, KIND_O, KIND_F,
                     KIND_M, KIND_COARSEST, KIND_CORR, KIND_LOOP)
from .noise import noise_vector, colour_masks, NOISE_Z4
from .dirac import gammas, gamma5
from .multigrid import gamma5_level


# ----------------------------------------------------------------- tr(D^-1)

def plain_samples(h, solvers, seed: int, nprobe: int, first: int = 0, noise: int = NOISE_Z4):
    n = h.ops[0].n
    out = np.zeros(nprobe, dtype=np.complex128)
    for k in range(nprobe):
        x = noise_vector(n, seed, stream_id(0, KIND_PLAIN), first + k, noise)
        out[k] = np.vdot(x, solvers[0](x))
    return out


def O_samples(h, solvers, l: int, seed: int, nprobe: int, first: int = 0, noise: int = NOISE_Z4):
    tr = h.transfers[l]
    n = h.ops[l].n
    out = np.zeros(nprobe, dtype=np.complex128)
    for k in range(nprobe):
        x = noise_vector(n, seed, stream_id(l, KIND_O), first + k, noise)
        y = tr.project_out(x)
        out[k] = np.vdot(y, solvers[l](y))
    return out


def F_samples(h, solvers, l: int, seed: int, nprobe: int, first: int = 0, noise: int = NOISE_Z4):
    tr = h.transfers[l]
    nc = h.ops[l + 1].n
    out = np.zeros(nprobe, dtype=np.complex128)
    for k in range(nprobe):
        x = noise_vector(nc, seed, stream_id(l, KIND_F), first + k, noise)
        px = tr.prolong(x)
        out[k] = np.vdot(px, solvers[l](px)) - np.vdot(x, solvers[l + 1](x))
    return out


def M_samples(h, solvers, l: int, seed: int, nprobe: int, first: int = 0, noise: int = NOISE_Z4):
    tr = h.transfers[l]
    n = h.ops[l].n
    out = np.zeros(nprobe, dtype=np.complex128)
    for k in range(nprobe):
        x = noise_vector(n, seed, stream_id(l, KIND_M), first + k, noise)
        xc = tr.restrict(x)
        out[k] = np.vdot(x, solvers[l](x)) - np.vdot(xc, solvers[l + 1](xc))
    return out


def coarsest_samples(h, solvers, seed: int, nprobe: int, first: int = 0, noise: int = NOISE_Z4):
    L = h.L
    n = h.ops[L - 1].n
    out = np.zeros(nprobe, dtype=np.complex128)
    for k in range(nprobe):
        x = noise_vector(n, seed, stream_id(L - 1, KIND_COARSEST), first + k, noise)
        out[k] = np.vdot(x, solvers[L - 1](x))
    return out


def mean_var(X: np.ndarray):
    """Sample mean and the paper's variance estimator sum|X - mu|^2/(N-1)."""
    X = np.asarray(X)
    mu = X.mean()
    var = float(np.sum(np.abs(X - mu) ** 2) / (len(X) - 1)) if len(X) > 1 else 0.0
    return mu, var


# ------------------------------------------------------------ exact (dense)

def offdiag_fro2(A: np.ndarray) -> float:
    """||offdiag(A)||_F^2: the Z4 Hutchinson variance times N (eq.
    variance-Frobenius-Relation)."""
    return float(np.sum(np.abs(A) ** 2) - np.sum(np.abs(np.diag(A)) ** 2))


def exact_operators(h):
    """Dense D_l^-1, P_l, and the MG-MLMC difference operators (small L)."""
    Dinv = [np.linalg.inv(op.dense()) for op in h.ops]
    P = [tr.dense() for tr in h.transfers]
    out = {"Dinv": Dinv, "P": P, "O": [], "F": [], "M": []}
    for l, Pl in enumerate(P):
        n = Pl.shape[0]
        Pi = Pl @ Pl.conj().T
        Q = np.eye(n) - Pi
        out["O"].append(Q @ Dinv[l] @ Q)
        out["F"].append(Pl.conj().T @ Dinv[l] @ Pl - Dinv[l + 1])
        out["M"].append(Dinv[l] - Pl @ Dinv[l + 1] @ Pl.conj().T)
    return out


# ------------------------------------------------------------- correlator

def _slice_of_sites(dims) -> np.ndarray:
    X, Y, Z, T = dims
    return np.repeat(np.arange(T), X * Y * Z)


def _slice_mask(dims, t: int) -> np.ndarray:
    """Boolean mask over fine dof for time slice t."""
    return np.repeat(_slice_of_sites(dims) == t, 12)


def term_levels(L: int, decomposition: str):
    """Finest level each term touches, in term order."""
    if decomposition == "plain":
        return [0]
    if decomposition == "oblique":
        return list(range(L))
    if decomposition == "orthogonal":
        return list(range(L - 1)) + list(range(L - 1)) + [L - 1]
    raise ValueError(decomposition)


class TermOperators:
    """Applies B_r and B~_r (fine -> fine) by their definitions."""

    def __init__(self, h, solvers, decomposition: str):
        self.h = h
        self.s = solvers
        self.dec = decomposition
        self.levels = term_levels(h.L, decomposition)

    def _embed(self, v, level):
        return self.h.prolong_to_fine(v, level)

    def apply(self, r: int, eta: np.ndarray, tilde: bool) -> np.ndarray:
        h, s, L = self.h, self.s, self.h.L
        if self.dec == "plain":
            return s[0](eta)
        if self.dec == "oblique":
            l = r
            y = h.restrict_from_fine(eta, l)
            if l == L - 1:
                return self._embed(s[l](y), l)
            tr = h.transfers[l]
            v = s[l](y) - tr.prolong(s[l + 1](tr.restrict(y)))
            return self._embed(v, l)
        # orthogonal
        if r == 2 * L - 2:
            y = h.restrict_from_fine(eta, L - 1)
            return self._embed(s[L - 1](y), L - 1)
        if r < L - 1:       # J_l
            l = r
            y = h.restrict_from_fine(eta, l)
            tr = h.transfers[l]
            if tilde:
                v = s[l](tr.project_out(y))
            else:
                v = tr.project_out(s[l](y))
            return self._embed(v, l)
        l = r - (L - 1)      # K_l
        y = h.restrict_from_fine(eta, l)
        tr = h.transfers[l]
        pw = tr.prolong(s[l + 1](tr.restrict(y)))
        if tilde:
            v = s[l](tr.prolong(tr.restrict(y))) - pw
        else:
            z = s[l](y)
            v = tr.prolong(tr.restrict(z)) - pw
        return self._embed(v, l)


def correlator_samples(h, solvers, decomposition: str, group: int, seed: int,
                       nprobe: int, first: int = 0, noise: int = NOISE_Z4):
    """Per-probe X_rs(t) for the pairs whose finest level is `group`.

    Returns (pairs, X) with pairs a list of (r, s) and X of shape
    (nprobe, len(pairs), T)."""
    ops = TermOperators(h, solvers, decomposition)
    lv = ops.levels
    R = len(lv)
    pairs = [(r, s) for r in range(R) for s in range(R) if min(lv[r], lv[s]) == group]
    needed = sorted({t for p in pairs for t in p})
    dims = h.ops[0].dims
    T = dims[3]
    n = h.ops[0].n
    sl = _slice_of_sites(dims)
    X = np.zeros((nprobe, len(pairs), T), dtype=np.complex128)
    for k in range(nprobe):
        eta = noise_vector(n, seed, stream_id(group, KIND_CORR), first + k, noise)
        for tp in range(T):
            e = np.where(_slice_mask(dims, tp), eta, 0)
            Bv = {r: ops.apply(r, e, False) for r in needed}
            Bt = {r: (ops.apply(r, e, True) if decomposition == "orthogonal" else Bv[r])
                  for r in needed}
            for ip, (r, s) in enumerate(pairs):
                prod = (np.conj(Bt[s]) * Bv[r]).reshape(-1, 12).sum(axis=1)
                S = np.bincount(sl, weights=prod.real, minlength=T) + \
                    1j * np.bincount(sl, weights=prod.imag, minlength=T)
                X[k, ip] += np.roll(S, -tp) / T   # X(t) += S[(t+tp) % T]/T
    return pairs, X


def exact_correlator(h, decomposition: str):
    """G_rs(t) = (1/T) sum_t' tr(B_r(t+t',t') G5 B_s(t',t+t') G5) from dense
    term matrices (small lattices only).  Returns (R, R, T)."""
    E = exact_operators(h)
    L = h.L
    Dinv, P = E["Dinv"], E["P"]
    Phat = [np.eye(h.ops[0].n)]
    for l in range(L - 1):
        Phat.append(Phat[-1] @ P[l])
    Bs = []
    if decomposition == "plain":
        Bs = [Dinv[0]]
    elif decomposition == "oblique":
        for l in range(L - 1):
            Bs.append(Phat[l] @ (Dinv[l] - P[l] @ Dinv[l + 1] @ P[l].conj().T) @ Phat[l].conj().T)
        Bs.append(Phat[L - 1] @ Dinv[L - 1] @ Phat[L - 1].conj().T)
    else:
        for l in range(L - 1):
            Pi = P[l] @ P[l].conj().T
            J = (np.eye(Pi.shape[0]) - Pi) @ Dinv[l]
            Bs.append(Phat[l] @ J @ Phat[l].conj().T)
        for l in range(L - 1):
            Pi = P[l] @ P[l].conj().T
            K = Pi @ Dinv[l] - P[l] @ Dinv[l + 1] @ P[l].conj().T
            Bs.append(Phat[l] @ K @ Phat[l].conj().T)
        Bs.append(Phat[L - 1] @ Dinv[L - 1] @ Phat[L - 1].conj().T)
    dims = h.ops[0].dims
    T = dims[3]
    g5 = np.kron(np.ones(h.ops[0].V), np.kron(np.diag(gamma5()).real, np.ones(3)))
    G5 = np.diag(g5)
    idx = [np.nonzero(_slice_mask(dims, t))[0] for t in range(T)]
    R = len(Bs)
    G = np.zeros((R, R, T), dtype=np.complex128)
    for r in range(R):
        for s in range(R):
            for t in range(T):
                acc = 0.0
                for tp in range(T):
                    t1 = (t + tp) % T
                    Br = Bs[r][np.ix_(idx[t1], idx[tp])]
                    Bs_ = Bs[s][np.ix_(idx[tp], idx[t1])]
                    g1 = G5[np.ix_(idx[tp], idx[tp])]
                    g2 = G5[np.ix_(idx[t1], idx[t1])]
                    acc += np.trace(Br @ g1 @ Bs_ @ g2)
                G[r, s, t] = acc / T
    return G, Bs


# ----------------------------------------------------------------- loops

GAMMA_NAMES = ["1", "g5", "gx", "gy", "gz", "gt"]


def gamma_list() -> np.ndarray:
    g = gammas()
    return np.stack([np.eye(4, dtype=np.complex128), gamma5(), g[0], g[1], g[2], g[3]])


def loop_samples(h, solvers, decomposition: str, group: int, seed: int,
                 nprobe: int, first: int = 0, noise: int = NOISE_Z4, probing: int = 1):
    """X[k, term, Gamma, t] = sum_{x in t} eta(x)^H Gamma (B eta)(x) for the
    terms whose finest level is `group`.  With probing p > 1 the source is
    split into the p^4 colours of noise.py and X sums the colours' values
    (one application of B per colour).  Returns (terms, X)."""
    ops = TermOperators(h, solvers, decomposition)
    terms = [r for r, lv in enumerate(ops.levels) if lv == group]
    dims = h.ops[0].dims
    T = dims[3]
    n = h.ops[0].n
    sl = _slice_of_sites(dims)
    Gs = gamma_list()
    X = np.zeros((nprobe, len(terms), 6, T), dtype=np.complex128)
    masks = colour_masks(dims, probing) if probing > 1 else [np.ones(n, dtype=bool)]
    for k in range(nprobe):
        eta_full = noise_vector(n, seed, stream_id(group, KIND_LOOP), first + k, noise)
        for mask in masks:
            eta = np.where(mask, eta_full, 0)
            e4 = eta.reshape(-1, 4, 3)
            for it, r in enumerate(terms):
                b4 = ops.apply(r, eta, False).reshape(-1, 4, 3)
                for ig in range(6):
                    gb = np.einsum("st,vtc->vsc", Gs[ig], b4)
                    prod = np.sum(np.conj(e4) * gb, axis=(1, 2))
                    X[k, it, ig] += np.bincount(sl, weights=prod.real, minlength=T) + \
                        1j * np.bincount(sl, weights=prod.imag, minlength=T)
    return terms, X


# ------------------------------------------------------------------ MLMC

def mlmc_allocation(V, C, eps2: float) -> np.ndarray:
    """Optimal real-valued N_l for target variance eps2 (eq. MLMC-Nl)."""
    V = np.asarray(V, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    s = np.sum(np.sqrt(V * C))
    return np.sqrt(V / C) * s / eps2
