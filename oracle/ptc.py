"""Gauge-covariant parallel-transport convolution (PTC) network in FP64
(oracle; test infrastructure only).

The paper does not describe a learned preconditioner; the network follows the
reading recorded in the design notes for the learned-preconditioner form of
the hot path.  A channel is one colour-triplet field on the lattice; the
network input and output are spinors (4 spin channels x colour).  One layer
maps c_in channels to c_out channels by

    out_a(x) = sum_p sum_b W_p[a, b] (T_p in_b)(x)

over nine paths p: p = 0 the identity, p = 1 + mu the forward transport
(T_{+mu} psi)(x) = U_mu(x) psi(x + mu), p = 5 + mu the backward transport
(T_{-mu} psi)(x) = U_mu(x - mu)^H psi(x - mu), with the antiperiodic sign on
hops across the time boundary (as in the Dirac operator).  W_p is a complex
c_out x c_in matrix.  Layers are linear (no activation), so the network is a
gauge-covariant linear operator of range equal to its depth.

Training objective (reading): for input r and target e, the per-sample loss is
|N(r) - e|^2 / |e|^2, averaged over the batch.

Gradient convention: for a complex quantity z the gradient is reported as
dL/dRe(z) + i dL/dIm(z).  For out = w t this gives grad_w = grad_out conj(t)
and grad_t = conj(w) grad_out.

Parity status: pinned by (i) the Wilson-Dirac operator (c_sw = 0) written as
a one-layer network with spin-matrix weights, compared with the independently
pinned oracle operator; (ii) exact gauge equivariance; (iii) the adjoint
identity of each transport; (iv) central finite differences of the loss.
"""
from __future__ import annotations

import numpy as np

NPATH = 9


def _axis(mu: int) -> int:
    # field arrays are [batch, T, Z, Y, X, channel, colour]; mu = 0..3 is x, y, z, t
    return {0: 4, 1: 3, 2: 2, 3: 1}[mu]


class PTC:
    """Parallel transports on a fixed gauge field U [T, Z, Y, X, 4, 3, 3]."""

    def __init__(self, U: np.ndarray, antiperiodic_t: bool = True):
        self.U = np.asarray(U, dtype=np.complex128)
        self.antiperiodic_t = bool(antiperiodic_t)
        self.T = self.U.shape[0]

    def _shift(self, psi: np.ndarray, mu: int, k: int) -> np.ndarray:
        """psi(x + k mu) for k = +1 / -1, with the time-boundary sign."""
        ax = _axis(mu)
        out = np.roll(psi, -k, axis=ax)
        if mu == 3 and self.antiperiodic_t:
            idx = [slice(None)] * psi.ndim
            idx[ax] = self.T - 1 if k == 1 else 0
            out[tuple(idx)] *= -1.0
        return out

    def transport(self, psi: np.ndarray, p: int) -> np.ndarray:
        """T_p psi for psi [batch, T, Z, Y, X, C, 3]."""
        if p == 0:
            return psi.copy()
        mu = (p - 1) % 4
        Um = self.U[..., mu, :, :]  # [T, Z, Y, X, 3, 3]
        if p <= 4:
            nb = self._shift(psi, mu, +1)
            return np.einsum("tzyxab,ntzyxcb->ntzyxca", Um, nb)
        # U_mu(x - mu)^H psi(x - mu)
        Ub = np.roll(Um, 1, axis=_axis(mu) - 1)
        nb = self._shift(psi, mu, -1)
        return np.einsum("tzyxba,ntzyxcb->ntzyxca", np.conj(Ub), nb)

    def transport_adj(self, phi: np.ndarray, p: int) -> np.ndarray:
        """T_p^H phi, written out from the definition of T_p: the forward
        transport's adjoint moves phi back along -mu with U^H, and vice versa."""
        if p == 0:
            return phi.copy()
        mu = (p - 1) % 4
        Um = self.U[..., mu, :, :]
        if p <= 4:
            # <T psi, phi> = sum_x phi(x)^H U(x) psi(x+mu)  =>  (T^H phi)(y) = U(y-mu)^H phi(y-mu)
            Ub = np.roll(Um, 1, axis=_axis(mu) - 1)
            nb = self._shift(phi, mu, -1)
            return np.einsum("tzyxba,ntzyxcb->ntzyxca", np.conj(Ub), nb)
        # <T psi, phi> = sum_x phi(x)^H U(x-mu)^H psi(x-mu)  =>  (T^H phi)(y) = U(y) phi(y+mu)
        nb = self._shift(phi, mu, +1)
        return np.einsum("tzyxab,ntzyxcb->ntzyxca", Um, nb)

    def layer(self, W: np.ndarray, psi: np.ndarray) -> np.ndarray:
        """sum_p W_p T_p psi; W [9, c_out, c_in]."""
        out = None
        for p in range(NPATH):
            t = np.einsum("ab,ntzyxbc->ntzyxac", W[p], self.transport(psi, p))
            out = t if out is None else out + t
        return out

    def forward(self, weights: list, r: np.ndarray) -> list:
        """Activations [r, h1, ..., out] for the layer weights list."""
        acts = [np.asarray(r, dtype=np.complex128)]
        for W in weights:
            acts.append(self.layer(W, acts[-1]))
        return acts

    def apply(self, weights: list, r: np.ndarray) -> np.ndarray:
        return self.forward(weights, r)[-1]

    def backward(self, weights: list, r: np.ndarray, g_out: np.ndarray):
        """Given dL/d(out) (complex convention), return (dL/dr, [dL/dW_l])."""
        acts = self.forward(weights, r)
        g = np.asarray(g_out, dtype=np.complex128)
        grads = [None] * len(weights)
        for l in range(len(weights) - 1, -1, -1):
            W, x = weights[l], acts[l]
            gW = np.zeros_like(W)
            gx = np.zeros_like(x)
            for p in range(NPATH):
                tp = self.transport(x, p)
                # grad_W[a, b] = sum over sites, colours, batch of g_a conj(t_b)
                gW[p] = np.einsum("ntzyxac,ntzyxbc->ab", g, np.conj(tp))
                # grad_t = W^H g, then back through the transport
                gt = np.einsum("ab,ntzyxac->ntzyxbc", np.conj(W[p]), g)
                gx += self.transport_adj(gt, p)
            grads[l] = gW
            g = gx
        return g, grads

    def loss(self, weights: list, r: np.ndarray, e: np.ndarray) -> float:
        out = self.apply(weights, r)
        n = r.shape[0]
        d = (out - e).reshape(n, -1)
        ee = np.asarray(e).reshape(n, -1)
        return float(np.mean(np.sum(np.abs(d) ** 2, axis=1) / np.sum(np.abs(ee) ** 2, axis=1)))

    def loss_grad(self, weights: list, r: np.ndarray, e: np.ndarray):
        """Loss and its gradients with respect to every layer's weights."""
        out = self.apply(weights, r)
        n = r.shape[0]
        d = out - e
        e2 = np.sum(np.abs(np.asarray(e).reshape(n, -1)) ** 2, axis=1)
        l = float(np.mean(np.sum(np.abs(d.reshape(n, -1)) ** 2, axis=1) / e2))
        scale = (2.0 / (n * e2)).reshape((n,) + (1,) * (d.ndim - 1))
        _, grads = self.backward(weights, r, scale * d)
        return l, grads


def wilson_weights(m0: float) -> list:
    """One 4 -> 4 layer equal to the Wilson-Dirac operator (c_sw = 0):
    W_0 = (4 + m0) 1, W_{+mu} = -(1 - g_mu)/2, W_{-mu} = -(1 + g_mu)/2,
    acting on the spin index (channel = spin)."""
    from .dirac import gammas
    g = gammas()
    I4 = np.eye(4, dtype=np.complex128)
    W = np.zeros((NPATH, 4, 4), dtype=np.complex128)
    W[0] = (4.0 + m0) * I4
    for mu in range(4):
        W[1 + mu] = -0.5 * (I4 - g[mu])
        W[5 + mu] = -0.5 * (I4 + g[mu])
    return [W]


def random_weights(widths, seed: int, scale: float = None) -> list:
    """Complex Gaussian weights for channel widths [c0, c1, ..., cL]."""
    rng = np.random.default_rng(seed)
    out = []
    for l in range(len(widths) - 1):
        ci, co = widths[l], widths[l + 1]
        s = scale if scale is not None else 1.0 / np.sqrt(NPATH * ci)
        out.append(s * (rng.standard_normal((NPATH, co, ci)) + 1j * rng.standard_normal((NPATH, co, ci)))
                   / np.sqrt(2.0))
    return out


def spinor_to_channels(psi: np.ndarray) -> np.ndarray:
    """[batch, T, Z, Y, X, 4, 3] spinors are already channel-major (spin = channel)."""
    return np.asarray(psi)
