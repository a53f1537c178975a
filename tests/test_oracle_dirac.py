"""Pins of the oracle's Wilson-clover operator (no GPU)."""
import numpy as np
import pytest

from lattice_inputs import gauge_field, unit_gauge, random_spinor, random_su3
from oracle.dirac import (WilsonClover, gammas, gamma5, sigma, field_strength,
                          free_field_trace_inverse, gamma5_vec)


def test_gamma_algebra():
    g = gammas()
    I4 = np.eye(4)
    for mu in range(4):
        np.testing.assert_allclose(g[mu], g[mu].conj().T, atol=0)
        for nu in range(4):
            ac = g[mu] @ g[nu] + g[nu] @ g[mu]
            np.testing.assert_allclose(ac, 2 * I4 * (mu == nu), atol=1e-15)
    np.testing.assert_allclose(gamma5(), np.diag([1, 1, -1, -1]), atol=1e-15)
    # sigma commutes with gamma5 (clover is chirality block diagonal)
    for mu in range(4):
        for nu in range(4):
            s = sigma(mu, nu)
            np.testing.assert_allclose(s, s.conj().T, atol=1e-15)
            np.testing.assert_allclose(s @ gamma5(), gamma5() @ s, atol=1e-15)


@pytest.mark.parametrize("dims,m0", [((2, 2, 2, 4), 0.2), ((4, 4, 2, 2), 0.05), ((2, 2, 4, 6), 0.5)])
def test_free_field_trace_closed_form(dims, m0):
    D = WilsonClover(unit_gauge(dims), m0, 1.0)
    Dinv = np.linalg.inv(D.dense())
    assert abs(np.trace(Dinv) - free_field_trace_inverse(dims, m0)) < 1e-11 * abs(np.trace(Dinv))


def test_free_field_periodic_time_differs():
    dims = (2, 2, 2, 4)
    D = WilsonClover(unit_gauge(dims), 0.3, 0.0, antiperiodic_t=False)
    tr = np.trace(np.linalg.inv(D.dense()))
    assert abs(tr - free_field_trace_inverse(dims, 0.3, antiperiodic_t=False)) < 1e-11 * abs(tr)
    assert abs(tr - free_field_trace_inverse(dims, 0.3, True)) > 1e-3


def test_plane_wave_eigenvectors():
    """For U = 1, e^{ipx} u is mapped to D(p) u with
    D(p) = m0 + sum(1 - cos p) + i sum g_mu sin p_mu."""
    dims = (4, 2, 2, 6)
    X, Y, Z, T = dims
    m0 = 0.1
    D = WilsonClover(unit_gauge(dims), m0, 0.0)
    n = (1, 0, 1, 2)
    p = [2 * np.pi * n[0] / X, 2 * np.pi * n[1] / Y, 2 * np.pi * n[2] / Z, (2 * n[3] + 1) * np.pi / T]
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    rng = np.random.default_rng(3)
    u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    psi = phase[..., None, None] * u
    g = gammas()
    Dp = (m0 + sum(1 - np.cos(q) for q in p)) * np.eye(4) + 1j * sum(g[mu] * np.sin(p[mu]) for mu in range(4))
    want = phase[..., None, None] * (Dp @ u)
    np.testing.assert_allclose(D.apply(psi), want, atol=1e-13)


def test_clover_vanishes_for_unit_links():
    F = field_strength(unit_gauge((2, 2, 2, 2)))
    assert np.abs(F).max() == 0.0


def test_single_link_field_strength_by_hand():
    """Only U_mu(x0) = V != 1.  Every plaquette leaf through that link equals
    V (traversed forward) or V^H (backward).  At x0 and x0+mu both leaves of
    the (mu,nu) plane appear, so F_mu_nu = 0 there; at x0+nu and x0+mu+nu a
    single forward leaf gives F = (V - V^H)/8, at x0-nu and x0+mu-nu a single
    backward leaf gives F = (V^H - V)/8."""
    dims = (4, 4, 4, 4)
    U = unit_gauge(dims)
    V = random_su3((), 0.7, np.random.default_rng(1))
    mu = 1
    x0 = (1, 2, 0, 3)  # x, y, z, t

    def idx(c):
        c = [c[i] % dims[i] for i in range(4)]
        return (c[3], c[2], c[1], c[0])

    U[idx(x0) + (mu,)] = V
    F = field_strength(U)
    A = (V - V.conj().T) / 8
    e = np.eye(4, dtype=int)
    for nu in range(4):
        if nu == mu:
            continue
        expect = {}
        expect[tuple(np.array(x0))] = 0
        expect[tuple(np.array(x0) + e[mu])] = 0
        expect[tuple(np.array(x0) + e[nu])] = A
        expect[tuple(np.array(x0) + e[mu] + e[nu])] = A
        expect[tuple(np.array(x0) - e[nu])] = -A
        expect[tuple(np.array(x0) + e[mu] - e[nu])] = -A
        for c, val in expect.items():
            np.testing.assert_allclose(F[mu, nu][idx(c)], val, atol=1e-15)
            np.testing.assert_allclose(F[nu, mu][idx(c)], -np.asarray(val), atol=1e-15)
        # all other sites zero in this plane
        mask = np.ones(F.shape[2:6], bool)
        for c in expect:
            mask[idx(c)] = False
        assert np.abs(F[mu, nu][mask]).max() < 1e-15


def test_single_link_clover_block_by_hand():
    """At x0+nu only the (mu,nu) plane is non-zero, so the local block is
    (4+m0) + c_sw (i/4) * 2 sigma_mu_nu (x) (V - V^H)/8."""
    dims = (4, 4, 4, 4)
    U = unit_gauge(dims)
    V = random_su3((), 0.7, np.random.default_rng(2))
    mu, nu, m0, csw = 0, 2, 0.3, 1.7
    x0 = (2, 1, 1, 0)
    U[(x0[3], x0[2], x0[1], x0[0], mu)] = V
    D = WilsonClover(U, m0, csw)
    site = (x0[3], x0[2] + 1, x0[1], x0[0])  # x0 + z-hat
    want = (4 + m0) * np.eye(12) + csw * 0.25j * 2 * np.kron(sigma(mu, nu), (V - V.conj().T) / 8)
    blocks, _ = D.stencil()
    X, Y, Z, T = dims
    s = x0[0] + X * (x0[1] + Y * ((x0[2] + 1) + Z * x0[3]))
    np.testing.assert_allclose(blocks[s, 0], want, atol=1e-14)


@pytest.fixture(scope="module")
def rough():
    U = gauge_field((4, 4, 4, 4), 0.5, 12)
    return U, WilsonClover(U, 0.05, 1.0)


def test_gamma5_hermiticity(rough):
    _, D = rough
    rng = np.random.default_rng(0)
    x = rng.standard_normal(D.n) + 1j * rng.standard_normal(D.n)
    y = rng.standard_normal(D.n) + 1j * rng.standard_normal(D.n)
    a = np.vdot(x, gamma5_vec(D.matvec(y)))
    b = np.conj(np.vdot(y, gamma5_vec(D.matvec(x))))
    assert abs(a - b) < 1e-12 * abs(a)
    Dd = D.dense()
    g5 = np.tile(np.repeat([1.0, 1.0, -1.0, -1.0], 3), D.V)
    np.testing.assert_allclose(g5[:, None] * Dd * g5[None, :], Dd.conj().T, atol=1e-14)


def test_gauge_covariance(rough):
    U, D = rough
    G = random_su3(U.shape[:4], 1.0, np.random.default_rng(5))
    Ug = U.copy()
    for mu in range(4):
        ax = {0: 3, 1: 2, 2: 1, 3: 0}[mu]
        Ug[..., mu, :, :] = G @ U[..., mu, :, :] @ np.roll(G, -1, axis=ax).conj().swapaxes(-1, -2)
    Dg = WilsonClover(Ug, D.m0, D.csw)
    psi = random_spinor((4, 4, 4, 4), 3)
    lhs = Dg.apply(np.einsum("...ab,...sb->...sa", G, psi))
    rhs = np.einsum("...ab,...sb->...sa", G, D.apply(psi))
    np.testing.assert_allclose(lhs, rhs, atol=1e-13)


def test_stencil_matches_apply_and_batches(rough):
    _, D = rough
    x = random_spinor((4, 4, 4, 4), 9, batch=2).reshape(2, -1)
    Dd = D.dense()
    np.testing.assert_allclose(D.matvec(x), x @ Dd.T, atol=1e-13)


def test_wilson_without_clover_is_gamma5_hermitian_odd_shape():
    dims = (2, 4, 2, 6)
    D = WilsonClover(gauge_field(dims, 0.3, 1), 0.2, 0.0)
    Dd = D.dense()
    g5 = np.tile(np.repeat([1.0, 1.0, -1.0, -1.0], 3), D.V)
    np.testing.assert_allclose(g5[:, None] * Dd * g5[None, :], Dd.conj().T, atol=1e-14)
