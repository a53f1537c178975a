"""Aggregation-based multigrid hierarchy in FP64 (oracle; test infrastructure).

What the paper fixes (Sec. 2.2): aggregation-based, adaptive transfer
operators with R_l = P_l^H and unitary P_l (P_l^H P_l = I); the Galerkin coarse
operator D_{l+1} = R_l D_l P_l; P_l built from N_tv test vectors that roughly
approximate the low modes of D_l (residual about 1e-1, Sec. 4).  What it leaves
open, and the readings used here (also recorded in the design notes):

* Aggregates are b^4 blocks of sites (b per direction may differ); a coarse
  site is an aggregate, numbered lexicographically like fine sites.
* Every level has d dof per site split into two chiralities of d/2 each:
  fine dof = 3*spin + colour = 6*chi + j; coarse dof = N_tv*chi + k.
  P is block diagonal per (aggregate, chirality); block row index is
  loc*(d/2) + j with loc the lexicographic site index inside the aggregate.
  Hence Gamma5 P = P Gamma5_c (Gamma5_c = +1 on chi = 0, -1 on chi = 1).
* Test vectors: v = Z4 probe (kind 7); 20 times: v <- MR_4(D_l, v),
  v <- v / |v|, where MR_4 runs 4 minimal-residual steps on D_l y = v from 0.
  Optionally (Sec. 5, more accurate test vectors) the fine level's vectors
  are refined to a target eigen-residual (refine_test_vectors).
* Orthonormalisation: modified Gram-Schmidt with one re-orthogonalisation
  pass per (aggregate, chirality) block, columns in order; diag(R) > 0 so the
  result is unique.  A column whose norm falls below 1e-12 of its original
  norm makes the block rank deficient.
* Coarse operator: nine-point stencil A[s_c, dir] (dir 0 self, 1+mu forward,
  5+mu backward), assembled hop by hop from the fine nine-point form.  This is
  D_c = P^H D P regrouped by which aggregate each fine hop lands in; it is
  compared with the dense product on small lattices.

Parity status: aggregation maps pinned bit-exactly by hand-countable cases;
P pinned by P^H P = I, sparsity and Gamma5 commutation; D_c pinned by the
dense P^H D P and by Gamma5_c-hermiticity.
"""
from __future__ import annotations

import numpy as np

from .dirac import WilsonClover, stencil_dense
from .philox import z4_vector, stream_id, KIND_TV


class RankDeficient(RuntimeError):
    pass


class Aggregation:
    """Maps between a lattice with d dof per site and its aggregates."""

    def __init__(self, dims, block, dof: int):
        self.dims = tuple(int(v) for v in dims)  # X, Y, Z, T
        self.block = tuple(int(v) for v in block)
        self.dof = int(dof)
        for L, b in zip(self.dims, self.block):
            if b < 1 or L % b != 0 or L // b < 2:
                raise ValueError("lattice %s not divisible into blocks %s with "
                                 "coarse extent >= 2" % (self.dims, self.block))
        self.cdims = tuple(L // b for L, b in zip(self.dims, self.block))
        self.V = int(np.prod(self.dims))
        self.Vc = int(np.prod(self.cdims))
        self.bvol = int(np.prod(self.block))
        self.half = self.dof // 2
        self.rows = self.bvol * self.half
        X, Y, Z, T = self.dims
        t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y),
                                 np.arange(X), indexing="ij")
        c = [x // self.block[0], y // self.block[1], z // self.block[2], t // self.block[3]]
        l = [x % self.block[0], y % self.block[1], z % self.block[2], t % self.block[3]]
        cx, cy, cz, ct = self.cdims
        bx, by, bz, bt = self.block
        self.agg = (c[0] + cx * (c[1] + cy * (c[2] + cz * c[3]))).reshape(-1)
        self.loc = (l[0] + bx * (l[1] + by * (l[2] + bz * l[3]))).reshape(-1)

    def block_index(self) -> np.ndarray:
        """perm[a, chi, row] = flat fine dof index (s*d + chi*half + j),
        row = loc*half + j.  Shape (Vc, 2, rows), int64."""
        perm = np.zeros((self.Vc, 2, self.rows), dtype=np.int64)
        s = np.arange(self.V)
        for chi in range(2):
            for j in range(self.half):
                perm[self.agg, chi, self.loc * self.half + j] = s * self.dof + chi * self.half + j
        return perm

    def to_blocks(self, v: np.ndarray) -> np.ndarray:
        """[..., n] -> [..., Vc, 2, rows]"""
        return v[..., self.block_index()]

    def from_blocks(self, vb: np.ndarray) -> np.ndarray:
        out = np.zeros(vb.shape[:-3] + (self.V * self.dof,), dtype=vb.dtype)
        out[..., self.block_index()] = vb
        return out


def mr_steps(apply, v: np.ndarray, steps: int) -> np.ndarray:
    """Minimal-residual iteration for D y = v from y = 0:
    r = v - D y, q = D r, alpha = q^H r / q^H q, y += alpha r, r -= alpha q."""
    y = np.zeros_like(v)
    r = v.copy()
    for _ in range(steps):
        q = apply(r)
        alpha = np.vdot(q, r) / np.vdot(q, q).real
        y = y + alpha * r
        r = r - alpha * q
    return y


def test_vectors(apply, n: int, ntv: int, seed: int, level: int,
                 setup_steps: int = 20, mr: int = 4) -> np.ndarray:
    """N_tv rough low modes of D_l, shape (ntv, n)."""
    out = np.zeros((ntv, n), dtype=np.complex128)
    for k in range(ntv):
        v = z4_vector(n, seed, stream_id(level, KIND_TV), k)
        for _ in range(setup_steps):
            y = mr_steps(apply, v, mr)
            v = y / np.linalg.norm(y)
        out[k] = v
    return out


def refine_test_vectors(apply, solve, V0: np.ndarray, max_iters: int, eig_tol: float):
    """Higher-accuracy test vectors of the fine operator (Sec. 5: test vectors
    with eigen-residuals down to 1e-4 give a stronger coarse space).

    Reading: inverse block power on the Hermitian Q = Gamma5 D with a
    Rayleigh-Ritz step after every QR.  V0 (n x k) are the rough test vectors;
    V = QR(V0); then, until every Ritz pair has
    rho_i = |Q v_i - theta_i v_i| / |theta_i| <= eig_tol or max_iters power
    steps are done: Rayleigh-Ritz (H = V^H Q V = S diag(theta) S^H, Ritz values
    ordered by |theta| ascending, V <- V S, each column's phase fixed so that
    the sum of its entries is real and positive), then a power step
    V <- QR(D^-1 Gamma5 V).  QR is modified Gram-Schmidt with one
    re-orthogonalisation pass and positive diag(R).  Returns (V, rho, steps)."""
    from .deflation import mgs2, gamma5_fine

    V = mgs2(V0)
    steps = 0
    while True:
        DV = np.stack([apply(V[:, j]) for j in range(V.shape[1])], axis=1)
        G5V = np.stack([gamma5_fine(V[:, j]) for j in range(V.shape[1])], axis=1)
        H = G5V.conj().T @ DV
        H = 0.5 * (H + H.conj().T)
        theta, S = np.linalg.eigh(H)
        order = np.argsort(np.abs(theta), kind="stable")
        theta, S = theta[order], S[:, order]
        V = V @ S
        QV = np.stack([gamma5_fine(c) for c in (DV @ S).T], axis=1)
        rho = np.linalg.norm(QV - V * theta[None, :], axis=0) / np.abs(theta)
        s = V.sum(axis=0)
        V = V * (np.conj(s) / np.abs(s))[None, :]
        if rho.max() <= eig_tol or steps >= max_iters:
            return V, rho, steps
        W = np.stack([solve(gamma5_fine(V[:, j])) for j in range(V.shape[1])], axis=1)
        V = mgs2(W)
        steps += 1


def block_mgs2(Vb: np.ndarray) -> np.ndarray:
    """Orthonormalise the columns of every block.

    Vb: (..., rows, ntv).  Modified Gram-Schmidt over columns in order with one
    re-orthogonalisation pass; returns Q with the same shape."""
    Q = np.zeros_like(Vb)
    ntv = Vb.shape[-1]
    for k in range(ntv):
        w = Vb[..., k].copy()
        n0 = np.linalg.norm(w, axis=-1)
        for _ in range(2):
            for j in range(k):
                h = np.sum(np.conj(Q[..., j]) * w, axis=-1)
                w = w - h[..., None] * Q[..., j]
        nrm = np.linalg.norm(w, axis=-1)
        if np.any(nrm < 1e-12 * n0) or np.any(n0 == 0):
            raise RankDeficient("test-vector block is rank deficient at column %d" % k)
        Q[..., k] = w / nrm[..., None]
    return Q


class Transfer:
    """P_l as blocks P[a, chi, row, k] and its action on flat vectors."""

    def __init__(self, agg: Aggregation, P: np.ndarray):
        self.agg = agg
        self.P = P  # (Vc, 2, rows, ntv)
        self.ntv = P.shape[-1]
        self.nc = agg.Vc * 2 * self.ntv
        self.perm = agg.block_index()

    def restrict(self, v: np.ndarray) -> np.ndarray:
        """P^H v: [..., n] -> [..., nc] with coarse dof = (a*2 + chi)*ntv + k."""
        vb = v[..., self.perm]  # (..., Vc, 2, rows)
        vc = np.einsum("acrk,...acr->...ack", np.conj(self.P), vb)
        return vc.reshape(vc.shape[:-3] + (self.nc,))

    def prolong(self, vc: np.ndarray) -> np.ndarray:
        """P vc: [..., nc] -> [..., n]."""
        a = self.agg
        vcb = vc.reshape(vc.shape[:-1] + (a.Vc, 2, self.ntv))
        vb = np.einsum("acrk,...ack->...acr", self.P, vcb)
        out = np.zeros(vc.shape[:-1] + (a.V * a.dof,), dtype=np.complex128)
        out[..., self.perm] = vb
        return out

    def project_out(self, v: np.ndarray) -> np.ndarray:
        """(I - P P^H) v, the orthogonal projector onto range(P)^perp."""
        return v - self.prolong(self.restrict(v))

    def dense(self) -> np.ndarray:
        """P as an n x nc matrix (small lattices only)."""
        return self.prolong(np.eye(self.nc, dtype=np.complex128)).T.copy()

    def site_matrices(self) -> np.ndarray:
        """Pfull[s] = rows of P belonging to fine site s: (V, d, 2*ntv)."""
        a = self.agg
        out = np.zeros((a.V, a.dof, 2 * self.ntv), dtype=np.complex128)
        for chi in range(2):
            for j in range(a.half):
                out[:, chi * a.half + j, chi * self.ntv:(chi + 1) * self.ntv] = \
                    self.P[a.agg, chi, a.loc * a.half + j, :]
        return out


class StencilOperator:
    """A level operator given by a nine-point stencil of dense d x d blocks."""

    def __init__(self, blocks: np.ndarray, nbr: np.ndarray, dims):
        self.blocks = blocks  # (V, 9, d, d)
        self.nbr = nbr        # (9, V)
        self.dims = tuple(dims)
        self.V = blocks.shape[0]
        self.d = blocks.shape[-1]
        self.n = self.V * self.d

    def matvec(self, x: np.ndarray) -> np.ndarray:
        xs = x.reshape(x.shape[:-1] + (self.V, self.d))
        y = np.zeros_like(xs)
        for k in range(self.blocks.shape[1]):
            y = y + np.einsum("sij,...sj->...si", self.blocks[:, k], xs[..., self.nbr[k], :])
        return y.reshape(x.shape)

    def stencil(self):
        return self.blocks, self.nbr

    def dense(self) -> np.ndarray:
        return stencil_dense(self.blocks, self.nbr)


def coarse_neighbours(cdims) -> np.ndarray:
    X, Y, Z, T = cdims
    V = X * Y * Z * T
    sites = np.arange(V).reshape(T, Z, Y, X)
    nbr = np.zeros((9, V), dtype=np.int64)
    nbr[0] = sites.reshape(-1)
    for mu in range(4):
        ax = {0: 3, 1: 2, 2: 1, 3: 0}[mu]
        nbr[1 + mu] = np.roll(sites, -1, axis=ax).reshape(-1)
        nbr[5 + mu] = np.roll(sites, 1, axis=ax).reshape(-1)
    return nbr


def galerkin(op, tr: Transfer) -> StencilOperator:
    """D_c = P^H D P as a nine-point coarse stencil.

    For every fine site x and stencil direction k with neighbour y, the block
    Pfull(x)^H B[x, k] Pfull(y) lands in A_c[agg(x), k] if the hop leaves the
    aggregate and in A_c[agg(x), 0] otherwise."""
    blocks, nbr = op.stencil()
    a = tr.agg
    Pf = tr.site_matrices()
    dc = 2 * tr.ntv
    A = np.zeros((a.Vc, 9, dc, dc), dtype=np.complex128)
    for k in range(9):
        y = nbr[k]
        M = np.einsum("sai,sab,sbj->sij", np.conj(Pf), blocks[:, k], Pf[y])
        target = np.where((k == 0) | (a.agg[y] == a.agg), 0, k)
        np.add.at(A, (a.agg, target), M)
    return StencilOperator(A, coarse_neighbours(a.cdims), a.cdims)


class Hierarchy:
    """Levels D_0 (fine) .. D_{L-1} and transfers P_0 .. P_{L-2}."""

    def __init__(self, fine, blocks, ntvs, seed: int, setup_steps: int = 20,
                 mr: int = 4, refine=None):
        """refine: None, or (solve, max_iters, eig_tol) to replace the level-0
        test vectors by refine_test_vectors(fine.matvec, solve, ...) of the
        rough ones (the coarser levels keep the rough recipe)."""
        self.ops = [fine]
        self.transfers = []
        self.tvs = []
        dims = fine.dims
        dof = 12
        for l, (b, ntv) in enumerate(zip(blocks, ntvs)):
            op = self.ops[-1]
            agg = Aggregation(dims, b, dof)
            tv = test_vectors(op.matvec, op.n, ntv, seed, l, setup_steps, mr)
            if l == 0 and refine is not None:
                solve, iters, tol = refine
                Vr, self.refine_rho, self.refine_steps = refine_test_vectors(op.matvec, solve, tv.T.copy(),
                                                                             iters, tol)
                tv = Vr.T.copy()
            self.tvs.append(tv)
            Vb = tv.T[agg.block_index()]       # (Vc, 2, rows, ntv)
            P = block_mgs2(Vb)
            tr = Transfer(agg, P)
            self.transfers.append(tr)
            self.ops.append(galerkin(op, tr))
            dims = agg.cdims
            dof = 2 * ntv

    @property
    def L(self) -> int:
        return len(self.ops)

    def prolong_to_fine(self, v: np.ndarray, level: int) -> np.ndarray:
        """P_hat_{level-1} v = P_0 ... P_{level-1} v."""
        for l in range(level - 1, -1, -1):
            v = self.transfers[l].prolong(v)
        return v

    def restrict_from_fine(self, v: np.ndarray, level: int) -> np.ndarray:
        """P_hat_{level-1}^H v."""
        for l in range(level):
            v = self.transfers[l].restrict(v)
        return v


def gamma5_level(n_sites: int, dof: int) -> np.ndarray:
    """Diagonal of Gamma5 on a level with dof per site: +1 on chi = 0."""
    g = np.ones((n_sites, 2, dof // 2))
    g[:, 1, :] = -1.0
    return g.reshape(-1)
