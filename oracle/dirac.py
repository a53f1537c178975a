"""Wilson-clover Dirac operator in FP64 (oracle; test infrastructure only).

The paper only says that D is the discretised Dirac operator on a 4-d lattice
with 12 degrees of freedom per site (4 spin x 3 colour, Sec. 1) and that it is
Gamma5-hermitian with a diagonal Gamma5 flipping half of the spin components
(Sec. 2.1, "Deflation for the Dirac operator").  The operator used here is the
standard Wilson-clover discretisation (reading recorded in the design notes):

  (D psi)(x) = (4 + m0) psi(x)
               - 1/2 sum_mu [ (1 - g_mu) U_mu(x) psi(x+mu)
                            + (1 + g_mu) U_mu(x-mu)^H psi(x-mu) ]
               + c_sw (i/4) sum_{mu != nu} sigma_mu_nu F_mu_nu(x) psi(x)

sigma_mu_nu = (i/2)[g_mu, g_nu], F_mu_nu = (Q_mu_nu - Q_mu_nu^H)/8 with Q the
sum of the four plaquette leaves at x, all oriented mu-then-nu.  Boundary
conditions: periodic in space, antiperiodic in time (the hop between t = T-1
and t = 0 carries a factor -1 in both directions); the clover term is built
from the unphased links.

Gamma basis (chiral, Euclidean): g_k = [[0, -i s_k], [i s_k, 0]] for
mu = x, y, z (k = 1, 2, 3) and g_t = [[0, 1], [1, 0]], so that
g5 = g_x g_y g_z g_t = diag(1, 1, -1, -1).

Parity status: pinned by the free-field closed form of tr D^-1, plane-wave
eigenvalues, Gamma5-hermiticity, gauge covariance and a single-link clover
configuration computed by hand (tests/test_oracle_dirac.py).
"""
from __future__ import annotations

import numpy as np

_s1 = np.array([[0, 1], [1, 0]], dtype=np.complex128)
_s2 = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
_s3 = np.array([[1, 0], [0, -1]], dtype=np.complex128)
_I2 = np.eye(2, dtype=np.complex128)
_Z2 = np.zeros((2, 2), dtype=np.complex128)


def _blk(a, b, c, d):
    return np.block([[a, b], [c, d]])


def gammas() -> np.ndarray:
    """g_mu for mu = 0..3 (x, y, z, t), shape (4, 4, 4)."""
    return np.stack([
        _blk(_Z2, -1j * _s1, 1j * _s1, _Z2),
        _blk(_Z2, -1j * _s2, 1j * _s2, _Z2),
        _blk(_Z2, -1j * _s3, 1j * _s3, _Z2),
        _blk(_Z2, _I2, _I2, _Z2),
    ])


def gamma5() -> np.ndarray:
    g = gammas()
    return g[0] @ g[1] @ g[2] @ g[3]


def sigma(mu: int, nu: int) -> np.ndarray:
    g = gammas()
    return 0.5j * (g[mu] @ g[nu] - g[nu] @ g[mu])


def _axis(mu: int) -> int:
    # arrays are [..., T, Z, Y, X, ...]; mu = 0..3 is x, y, z, t
    return {0: 3, 1: 2, 2: 1, 3: 0}[mu]


def _shift_links(A: np.ndarray, mu: int, k: int) -> np.ndarray:
    """A at x + k*mu for a link-type array [T, Z, Y, X, 3, 3] (periodic)."""
    return np.roll(A, -k, axis=_axis(mu))


def _dag(A: np.ndarray) -> np.ndarray:
    return np.conj(np.swapaxes(A, -1, -2))


def field_strength(U: np.ndarray) -> np.ndarray:
    """Clover-leaf F_mu_nu(x) for all mu, nu; shape (4, 4, T, Z, Y, X, 3, 3)."""
    F = np.zeros((4, 4) + U.shape[:4] + (3, 3), dtype=np.complex128)
    for mu in range(4):
        for nu in range(4):
            if mu == nu:
                continue
            Um = U[..., mu, :, :]
            Un = U[..., nu, :, :]
            S = _shift_links
            # leaf 1: x -> x+mu -> x+mu+nu -> x+nu -> x
            l1 = Um @ S(Un, mu, 1) @ _dag(S(Um, nu, 1)) @ _dag(Un)
            # leaf 2: x -> x+nu -> x+nu-mu -> x-mu -> x
            l2 = Un @ _dag(S(S(Um, nu, 1), mu, -1)) @ _dag(S(Un, mu, -1)) @ S(Um, mu, -1)
            # leaf 3: x -> x-mu -> x-mu-nu -> x-nu -> x
            l3 = (_dag(S(Um, mu, -1)) @ _dag(S(S(Un, mu, -1), nu, -1))
                  @ S(S(Um, mu, -1), nu, -1) @ S(Un, nu, -1))
            # leaf 4: x -> x-nu -> x-nu+mu -> x+mu -> x
            l4 = _dag(S(Un, nu, -1)) @ S(Um, nu, -1) @ S(S(Un, nu, -1), mu, 1) @ _dag(Um)
            Q = l1 + l2 + l3 + l4
            F[mu, nu] = (Q - _dag(Q)) / 8.0
    return F


def clover_matrix(U: np.ndarray, csw: float) -> np.ndarray:
    """Site-local clover term c_sw (i/4) sum_{mu!=nu} sigma_mu_nu (x) F_mu_nu.

    Shape (T, Z, Y, X, 12, 12) with dof index = 3 * spin + colour.
    """
    F = field_strength(U)
    C = np.zeros(U.shape[:4] + (12, 12), dtype=np.complex128)
    for mu in range(4):
        for nu in range(4):
            if mu == nu:
                continue
            s = sigma(mu, nu)
            C += np.einsum("st,...ab->...satb", s, F[mu, nu]).reshape(U.shape[:4] + (12, 12))
    return csw * 0.25j * C


class WilsonClover:
    """D[U] for fixed links; apply() works on [..., T, Z, Y, X, 4, 3] arrays."""

    def __init__(self, U: np.ndarray, m0: float, csw: float,
                 antiperiodic_t: bool = True):
        self.U = np.asarray(U, dtype=np.complex128)
        self.dims = (U.shape[3], U.shape[2], U.shape[1], U.shape[0])  # X, Y, Z, T
        self.m0 = float(m0)
        self.csw = float(csw)
        self.antiperiodic_t = bool(antiperiodic_t)
        self.g = gammas()
        self.clover = clover_matrix(self.U, self.csw) if csw != 0.0 else None
        self.V = int(np.prod(self.dims))
        self.n = 12 * self.V

    def _shift_psi(self, psi: np.ndarray, mu: int, k: int) -> np.ndarray:
        """psi(x + k*mu) with the time boundary phase, for k = +1 or -1."""
        ax = psi.ndim - 6 + _axis(mu)
        out = np.roll(psi, -k, axis=ax)
        if mu == 3 and self.antiperiodic_t:
            T = psi.shape[ax]
            idx = [slice(None)] * psi.ndim
            idx[ax] = T - 1 if k == 1 else 0
            out[tuple(idx)] *= -1.0
        return out

    def hop(self, psi: np.ndarray, mu: int, sign: int) -> np.ndarray:
        """One hopping term (without the -1/2):
        sign=+1: (1 - g_mu) U_mu(x) psi(x+mu)
        sign=-1: (1 + g_mu) U_mu(x-mu)^H psi(x-mu)."""
        I4 = np.eye(4, dtype=np.complex128)
        Um = self.U[..., mu, :, :]
        if sign > 0:
            link = Um
            proj = I4 - self.g[mu]
        else:
            link = _dag(_shift_links(Um, mu, -1))
            proj = I4 + self.g[mu]
        nb = self._shift_psi(psi, mu, sign)
        col = np.einsum("...ab,...sb->...sa", link, nb)
        return np.einsum("st,...ta->...sa", proj, col)

    def local(self, psi: np.ndarray) -> np.ndarray:
        out = (4.0 + self.m0) * psi
        if self.clover is not None:
            sh = psi.shape
            flat = psi.reshape(sh[:-2] + (12,))
            out = out + np.einsum("...ij,...j->...i", self.clover, flat).reshape(sh)
        return out

    def apply(self, psi: np.ndarray) -> np.ndarray:
        out = self.local(psi)
        for mu in range(4):
            out = out - 0.5 * (self.hop(psi, mu, +1) + self.hop(psi, mu, -1))
        return out

    # flat-vector interface: x of length 12 V (or [batch, 12 V])
    def matvec(self, x: np.ndarray) -> np.ndarray:
        X, Y, Z, T = self.dims
        sh = x.shape[:-1]
        return self.apply(x.reshape(sh + (T, Z, Y, X, 4, 3))).reshape(sh + (self.n,))

    def stencil(self):
        """Nine-point form of D: blocks[s, dir] (12 x 12) and nbr[dir, s] such
        that (D psi)(s) = sum_dir blocks[s, dir] psi(nbr[dir, s]).
        dir 0 is the site itself, 1 + mu the hop to s + mu, 5 + mu the hop to
        s - mu; boundary phases are folded into the blocks."""
        X, Y, Z, T = self.dims
        V = self.V
        I4 = np.eye(4, dtype=np.complex128)
        blocks = np.zeros((V, 9, 12, 12), dtype=np.complex128)
        loc = (4.0 + self.m0) * np.eye(12, dtype=np.complex128)
        blocks[:, 0] = loc
        if self.clover is not None:
            blocks[:, 0] += self.clover.reshape(V, 12, 12)
        nbr = np.zeros((9, V), dtype=np.int64)
        sites = np.arange(V).reshape(T, Z, Y, X)
        nbr[0] = sites.reshape(-1)
        tcoord = np.broadcast_to(np.arange(T)[:, None, None, None], (T, Z, Y, X)).reshape(-1)
        for mu in range(4):
            ax = _axis(mu)
            Um = self.U[..., mu, :, :]
            fwd_link = Um.reshape(V, 3, 3)
            bwd_link = _dag(_shift_links(Um, mu, -1)).reshape(V, 3, 3)
            nbr[1 + mu] = np.roll(sites, -1, axis=ax).reshape(-1)
            nbr[5 + mu] = np.roll(sites, 1, axis=ax).reshape(-1)
            ph_f = np.ones(V)
            ph_b = np.ones(V)
            if mu == 3 and self.antiperiodic_t:
                ph_f[tcoord == T - 1] = -1.0
                ph_b[tcoord == 0] = -1.0
            bf = np.einsum("st,vab->vsatb", I4 - self.g[mu], fwd_link).reshape(V, 12, 12)
            bb = np.einsum("st,vab->vsatb", I4 + self.g[mu], bwd_link).reshape(V, 12, 12)
            blocks[:, 1 + mu] = -0.5 * ph_f[:, None, None] * bf
            blocks[:, 5 + mu] = -0.5 * ph_b[:, None, None] * bb
        return blocks, nbr

    def dense(self) -> np.ndarray:
        """Dense n x n matrix assembled from the nine-point form (tiny lattices)."""
        blocks, nbr = self.stencil()
        return stencil_dense(blocks, nbr)


def stencil_dense(blocks: np.ndarray, nbr: np.ndarray) -> np.ndarray:
    V, ndir, d, _ = blocks.shape
    M = np.zeros((V * d, V * d), dtype=np.complex128)
    for s in range(V):
        for k in range(ndir):
            t = nbr[k, s]
            M[s * d:(s + 1) * d, t * d:(t + 1) * d] += blocks[s, k]
    return M


def gamma5_vec(x: np.ndarray) -> np.ndarray:
    """Gamma5 on a flat fine vector (dof = 3*spin + colour): +1 for spins 0,1."""
    sh = x.shape
    v = x.reshape(sh[:-1] + (-1, 4, 3)).copy()
    v[..., 2:, :] *= -1.0
    return v.reshape(sh)


def free_field_trace_inverse(dims, m0: float, antiperiodic_t: bool = True) -> float:
    """Closed form of tr D^-1 for U = 1 (plane waves diagonalise D):
    D(p) = a(p) + i sum_mu g_mu sin p_mu, a(p) = m0 + sum_mu (1 - cos p_mu),
    so tr D(p)^-1 = 12 a / (a^2 + sum_mu sin^2 p_mu) (4 spins x 3 colours)."""
    X, Y, Z, T = dims
    ps = [2 * np.pi * np.arange(L) / L for L in (X, Y, Z)]
    if antiperiodic_t:
        ps.append((2 * np.arange(T) + 1) * np.pi / T)
    else:
        ps.append(2 * np.pi * np.arange(T) / T)
    P = np.meshgrid(*ps, indexing="ij")
    a = m0 + sum(1 - np.cos(p) for p in P)
    s2 = sum(np.sin(p) ** 2 for p in P)
    return float(np.sum(12 * a / (a ** 2 + s2)))
