"""Pins of the FP64 PTC-network oracle against the Dirac operator, gauge
symmetry, adjointness and finite differences."""
import numpy as np

from lattice_inputs import gauge_field, random_su3
from oracle.dirac import WilsonClover
from oracle.ptc import NPATH, PTC, random_weights, wilson_weights

DIMS = (4, 4, 4, 4)


def _field(seed, batch, C, dims=DIMS):
    rng = np.random.default_rng(seed)
    X, Y, Z, T = dims
    sh = (batch, T, Z, Y, X, C, 3)
    return rng.standard_normal(sh) + 1j * rng.standard_normal(sh)


def _inner(a, b):
    return np.vdot(a.ravel(), b.ravel())


def test_one_layer_wilson_weights_equal_wilson_operator():
    # the Wilson-Dirac operator is a one-layer network with spin-matrix weights
    U = gauge_field(DIMS, 0.5, 31)
    m0 = 0.13
    net = PTC(U)
    psi = _field(1, 2, 4)
    got = net.apply(wilson_weights(m0), psi)
    D = WilsonClover(U, m0, 0.0)
    want = np.stack([D.apply(psi[i]) for i in range(2)])
    assert np.max(np.abs(got - want)) < 1e-12 * np.max(np.abs(want))


def test_wilson_weights_periodic_time_variant():
    U = gauge_field((2, 2, 2, 4), 0.4, 32)
    net = PTC(U, antiperiodic_t=False)
    psi = _field(2, 1, 4, dims=(2, 2, 2, 4))
    got = net.apply(wilson_weights(0.3), psi)
    want = WilsonClover(U, 0.3, 0.0, antiperiodic_t=False).apply(psi[0])
    assert np.max(np.abs(got[0] - want)) < 1e-12 * np.max(np.abs(want))


def test_transport_adjoint_identity():
    U = gauge_field(DIMS, 0.6, 33)
    net = PTC(U)
    a = _field(3, 1, 5)
    b = _field(4, 1, 5)
    for p in range(NPATH):
        lhs = _inner(net.transport(a, p), b)
        rhs = _inner(a, net.transport_adj(b, p))
        assert abs(lhs - rhs) < 1e-11 * abs(lhs)


def test_forward_and_backward_transports_are_mutual_adjoints():
    # T_{+mu}^H = T_{-mu}: checked on the transports themselves
    U = gauge_field(DIMS, 0.6, 34)
    net = PTC(U)
    a = _field(5, 1, 3)
    for mu in range(4):
        x = net.transport_adj(a, 1 + mu)
        y = net.transport(a, 5 + mu)
        assert np.max(np.abs(x - y)) < 1e-13


def test_gauge_equivariance():
    # N[U^g](G r) = G N[U](r) with U^g_mu(x) = G(x) U_mu(x) G(x+mu)^H
    U = gauge_field(DIMS, 0.6, 35)
    G = random_su3(DIMS[::-1], 1.0, np.random.default_rng(36))  # [T, Z, Y, X, 3, 3]
    Ug = np.empty_like(U)
    for mu in range(4):
        ax = {0: 3, 1: 2, 2: 1, 3: 0}[mu]
        Gs = np.roll(G, -1, axis=ax)
        Ug[..., mu, :, :] = G @ U[..., mu, :, :] @ np.conj(np.swapaxes(Gs, -1, -2))
    W = random_weights([4, 6, 5, 4], 37)
    r = _field(38, 2, 4)
    Gr = np.einsum("tzyxab,ntzyxcb->ntzyxca", G, r)
    lhs = PTC(Ug).apply(W, Gr)
    rhs = np.einsum("tzyxab,ntzyxcb->ntzyxca", G, PTC(U).apply(W, r))
    assert np.max(np.abs(lhs - rhs)) < 1e-12 * np.max(np.abs(rhs))


def test_linearity():
    U = gauge_field(DIMS, 0.6, 39)
    net = PTC(U)
    W = random_weights([4, 3, 4], 40)
    r1, r2 = _field(41, 1, 4), _field(42, 1, 4)
    a, b = 0.3 - 1.2j, -0.7 + 0.4j
    lhs = net.apply(W, a * r1 + b * r2)
    rhs = a * net.apply(W, r1) + b * net.apply(W, r2)
    assert np.max(np.abs(lhs - rhs)) < 1e-12 * np.max(np.abs(rhs))


def test_loss_gradient_matches_central_differences():
    U = gauge_field((2, 2, 2, 4), 0.6, 43)
    net = PTC(U)
    W = random_weights([4, 5, 4], 44)
    r = _field(45, 2, 4, dims=(2, 2, 2, 4))
    e = _field(46, 2, 4, dims=(2, 2, 2, 4))
    l0, grads = net.loss_grad(W, r, e)
    assert abs(l0 - net.loss(W, r, e)) < 1e-14 * l0
    rng = np.random.default_rng(47)
    h = 1e-6
    for _ in range(12):
        li = int(rng.integers(len(W)))
        idx = tuple(int(rng.integers(s)) for s in W[li].shape)
        for part, unit in (("re", 1.0), ("im", 1j)):
            Wp = [w.copy() for w in W]
            Wm = [w.copy() for w in W]
            Wp[li][idx] += unit * h
            Wm[li][idx] -= unit * h
            fd = (net.loss(Wp, r, e) - net.loss(Wm, r, e)) / (2 * h)
            an = grads[li][idx].real if part == "re" else grads[li][idx].imag
            assert abs(fd - an) < 1e-6 * max(1.0, abs(an)), (li, idx, part, fd, an)


def test_input_gradient_matches_central_differences():
    # dL/dr for L = Re <c, N(r)>: the backward pass with g_out = c
    U = gauge_field((2, 2, 2, 4), 0.5, 48)
    net = PTC(U)
    W = random_weights([4, 4, 4], 49)
    r = _field(50, 1, 4, dims=(2, 2, 2, 4))
    c = _field(51, 1, 4, dims=(2, 2, 2, 4))
    g_in, _ = net.backward(W, r, c)

    def L(x):
        return float(np.real(_inner(c, net.apply(W, x))))

    rng = np.random.default_rng(52)
    h = 1e-6
    for _ in range(8):
        idx = tuple(int(rng.integers(s)) for s in r.shape)
        for unit, part in ((1.0, "re"), (1j, "im")):
            rp, rm = r.copy(), r.copy()
            rp[idx] += unit * h
            rm[idx] -= unit * h
            fd = (L(rp) - L(rm)) / (2 * h)
            an = g_in[idx].real if part == "re" else g_in[idx].imag
            assert abs(fd - an) < 1e-6 * max(1.0, abs(an))
