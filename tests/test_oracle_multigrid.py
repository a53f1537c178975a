"""Pins of the oracle's aggregation, test vectors, block QR, P and D_c."""
import numpy as np
import pytest

from lattice_inputs import gauge_field
from oracle.dirac import WilsonClover
from oracle.multigrid import (Aggregation, Hierarchy, block_mgs2, mr_steps, refine_test_vectors,
                              gamma5_level, RankDeficient, test_vectors as tv_fn)
from oracle.solve import gmres, DenseSolver, level_solver, relative_residual


def test_aggregation_map_by_hand():
    # dims X=4, Y=2, Z=2, T=4 with blocks (2, 1, 1, 2): coarse dims (2, 2, 2, 2)
    a = Aggregation((4, 2, 2, 4), (2, 1, 1, 2), 12)
    assert a.cdims == (2, 2, 2, 2) and a.bvol == 4 and a.rows == 24

    def s(x, y, z, t):
        return x + 4 * (y + 2 * (z + 2 * t))

    def c(x, y, z, t):
        return x + 2 * (y + 2 * (z + 2 * t))

    # site (3, 1, 0, 3): coarse (1, 1, 0, 1), local (1, 0, 0, 1) -> loc 1 + 2*1 = 3
    assert a.agg[s(3, 1, 0, 3)] == c(1, 1, 0, 1)
    assert a.loc[s(3, 1, 0, 3)] == 3
    assert a.agg[s(0, 0, 1, 0)] == c(0, 0, 1, 0) and a.loc[s(0, 0, 1, 0)] == 0
    perm = a.block_index()
    # fine dof of (site (3,1,0,3), spin 2, colour 1): chi = 1, j = 0*3 + 1 = 1
    fine = s(3, 1, 0, 3) * 12 + 2 * 3 + 1
    assert perm[c(1, 1, 0, 1), 1, 3 * 6 + 1] == fine
    # a permutation of all dof
    assert np.array_equal(np.sort(perm.reshape(-1)), np.arange(a.V * 12))


def test_aggregation_rejects_bad_shapes():
    with pytest.raises(ValueError):
        Aggregation((4, 4, 4, 4), (4, 2, 2, 2), 12)  # coarse extent 1
    with pytest.raises(ValueError):
        Aggregation((4, 4, 4, 6), (2, 2, 2, 4), 12)  # not divisible


def test_block_mgs2_matches_qr_with_positive_diagonal():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((3, 2, 20, 5)) + 1j * rng.standard_normal((3, 2, 20, 5))
    Q = block_mgs2(A)
    for a in range(3):
        for c in range(2):
            q, r = np.linalg.qr(A[a, c])
            ph = np.diag(r) / np.abs(np.diag(r))
            q = q * ph[None, :]
            np.testing.assert_allclose(Q[a, c], q, atol=1e-13)


def test_block_mgs2_rank_deficient():
    rng = np.random.default_rng(1)
    A = rng.standard_normal((1, 1, 10, 3)) + 0j
    A[..., 2] = A[..., 0] * 2.0 - A[..., 1]
    with pytest.raises(RankDeficient):
        block_mgs2(A)


def test_mr_steps_scalar_operator_and_minimal_residual():
    v = np.array([1.0 + 2j, -0.5j, 3.0])
    y = mr_steps(lambda r: (2.0 - 1j) * r, v, 1)
    np.testing.assert_allclose(y, v / (2.0 - 1j), atol=1e-15)
    rng = np.random.default_rng(2)
    M = np.eye(6) * 3 + rng.standard_normal((6, 6)) * 0.3
    b = rng.standard_normal(6) + 0j
    y1 = mr_steps(lambda r: M @ r, b, 1)
    r1 = np.linalg.norm(b - M @ y1)
    for da in (1e-3, -1e-3, 1e-3j):
        alpha = (y1 / b)[0] + da  # y1 = alpha * b after one step
        assert np.linalg.norm(b - alpha * (M @ b)) >= r1


@pytest.fixture(scope="module")
def hier44():
    U = gauge_field((4, 4, 4, 4), 0.5, 12)
    D = WilsonClover(U, 0.05, 1.0)
    return D, Hierarchy(D, [(2, 2, 2, 2)], [8], seed=102)


def test_P_is_unitary_sparse_and_chiral(hier44):
    D, h = hier44
    tr = h.transfers[0]
    P = tr.dense()
    np.testing.assert_allclose(P.conj().T @ P, np.eye(P.shape[1]), atol=1e-14)
    # sparsity: row (s, chi) only couples to coarse dof of (agg(s), chi)
    a = tr.agg
    for s in (0, 17, 255):
        for dof in range(12):
            chi = dof // 6
            nz = np.nonzero(np.abs(P[s * 12 + dof]) > 0)[0]
            assert set(nz) <= set(range(a.agg[s] * 16 + chi * 8, a.agg[s] * 16 + chi * 8 + 8))
    g5 = gamma5_level(D.V, 12)
    g5c = gamma5_level(a.Vc, 16)
    np.testing.assert_allclose(g5[:, None] * P, P * g5c[None, :], atol=0)


def test_test_vectors_are_rough_low_modes(hier44):
    D, h = hier44
    tv = h.tvs[0]
    np.testing.assert_allclose(np.linalg.norm(tv, axis=1), 1.0, atol=1e-14)
    # Rayleigh quotients |D v| are well below the typical |D x|/|x|
    rng = np.random.default_rng(3)
    x = rng.standard_normal(D.n) + 1j * rng.standard_normal(D.n)
    typical = np.linalg.norm(D.matvec(x)) / np.linalg.norm(x)
    low = np.array([np.linalg.norm(D.matvec(v)) for v in tv])
    assert low.max() < 0.6 * typical


def test_galerkin_matches_dense_product(hier44):
    D, h = hier44
    P = h.transfers[0].dense()
    np.testing.assert_allclose(h.ops[1].dense(), P.conj().T @ D.dense() @ P, atol=1e-13)


def test_coarse_operator_gamma5_hermitian(hier44):
    _, h = hier44
    Dc = h.ops[1].dense()
    g = gamma5_level(h.ops[1].V, 16)
    np.testing.assert_allclose(g[:, None] * Dc * g[None, :], Dc.conj().T, atol=1e-14)


def test_coarse_backward_blocks_from_forward(hier44):
    """The stencil form of gamma5-hermiticity that the BF16 coarse layout
    relies on: the backward block at x is the chirality-signed conjugate
    transpose of the forward block at x - mu (Gamma5_c = diag(+1, -1) over
    the two chirality halves of a coarse site)."""
    _, h = hier44
    op = h.ops[1]
    B, nbr = op.stencil()
    d = op.d
    g = np.where(np.arange(d) < d // 2, 1.0, -1.0)
    for mu in range(4):
        xm = nbr[5 + mu]
        want = g[None, :, None] * np.conj(np.transpose(B[xm, 1 + mu], (0, 2, 1))) * g[None, None, :]
        np.testing.assert_allclose(B[:, 5 + mu], want, atol=1e-14)
        # and the forward neighbour of x - mu is x
        assert np.array_equal(nbr[1 + mu][xm], np.arange(op.V))


def test_three_level_odd_shape():
    """4x4x4x8 -> (2,2,2,2) blocks -> 2x2x2x4 -> (1,1,1,2) -> 2x2x2x2."""
    U = gauge_field((4, 4, 4, 8), 0.5, 21)
    D = WilsonClover(U, 0.1, 1.0)
    h = Hierarchy(D, [(2, 2, 2, 2), (1, 1, 1, 2)], [6, 4], seed=7)
    assert [op.n for op in h.ops] == [6144, 32 * 12, 16 * 8]
    P1 = h.transfers[1].dense()
    np.testing.assert_allclose(P1.conj().T @ P1, np.eye(P1.shape[1]), atol=1e-14)
    np.testing.assert_allclose(h.ops[2].dense(), P1.conj().T @ h.ops[1].dense() @ P1, atol=1e-13)
    Ph = h.transfers[0].dense() @ P1
    np.testing.assert_allclose(h.ops[2].dense(), Ph.conj().T @ D.dense() @ Ph, atol=1e-12)


def test_gmres_matches_dense_lu(hier44):
    D, h = hier44
    rng = np.random.default_rng(4)
    b = rng.standard_normal(D.n) + 1j * rng.standard_normal(D.n)
    x = gmres(D.matvec, b, tol=1e-12)
    assert relative_residual(D.matvec, x, b) <= 1e-12
    xd = DenseSolver(D.dense())(b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-10
    s = level_solver(h.ops[1])
    bc = rng.standard_normal(h.ops[1].n) + 0j
    assert relative_residual(h.ops[1].matvec, s(bc), bc) < 1e-13


def test_mr4_on_a_diagonal_operator_by_hand():
    """Four minimal-residual steps from y = 0 on D = diag(1, 2), worked out by
    hand with exact fractions: from v = (1, 1) the lengths are 3/5, 3/4, 3/5,
    3/4 and y = (99/100, 99/200); from v = (2, 1) they are 3/4, 3/5, 3/4, 3/5
    and y = (198/100, 99/200)."""
    d = np.array([1.0, 2.0])
    y = mr_steps(lambda v: d * v, np.array([1.0, 1.0], dtype=complex), 4)
    np.testing.assert_allclose(y, [0.99, 0.495], rtol=0, atol=1e-15)
    y = mr_steps(lambda v: d * v, np.array([2.0, 1.0], dtype=complex), 4)
    np.testing.assert_allclose(y, [1.98, 0.495], rtol=0, atol=1e-15)
    # three steps stop at y = (0.96, 0.51): the step count matters
    y3 = mr_steps(lambda v: d * v, np.array([1.0, 1.0], dtype=complex), 3)
    np.testing.assert_allclose(y3, [0.96, 0.51], rtol=0, atol=1e-15)


def test_test_vectors_round_count_and_stream_by_hand():
    """Test vectors of D = diag(1, 2) from a Z4 start s(1, 1) (seed 8 gives
    s = -1 on the test-vector stream of level 0, and no other stream or probe
    gives that start): MR_4 is homogeneous of degree one, so by the hand values
    above one round gives s(2, 1)/sqrt(5) and two rounds s(4, 1)/sqrt(17).  A
    wrong round count, MR step count, stream kind, level or probe index gives
    another vector."""
    from oracle.philox import z4_vector, stream_id, KIND_TV
    d = np.array([1.0, 2.0])
    seed = 8
    start = z4_vector(2, seed, stream_id(0, KIND_TV), 0)
    assert start[0] == start[1] == -1.0
    s = start[0]
    v1 = tv_fn(lambda v: d * v, 2, 1, seed, 0, setup_steps=1, mr=4)
    np.testing.assert_allclose(v1[0], s * np.array([2.0, 1.0]) / np.sqrt(5.0), atol=1e-15)
    v2 = tv_fn(lambda v: d * v, 2, 1, seed, 0, setup_steps=2, mr=4)
    np.testing.assert_allclose(v2[0], s * np.array([4.0, 1.0]) / np.sqrt(17.0), atol=1e-15)
    assert np.linalg.norm(tv_fn(lambda v: d * v, 2, 1, seed, 0, setup_steps=2, mr=3)[0] - v2[0]) > 1e-3


def _known_spectrum(n=48, k=4, seed=3):
    from oracle.deflation import gamma5_fine
    rng = np.random.default_rng(seed)
    W, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    mags = np.concatenate([[0.5, 0.6, 0.7, 0.8], np.linspace(1.6, 24.0, n - 4)])
    lam = mags * np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    Q = W @ np.diag(lam) @ W.conj().T
    Dm = np.stack([gamma5_fine(Q[:, j]) for j in range(n)], axis=1)
    return W, lam, Dm


def test_refined_test_vectors_converge_to_eigenpairs():
    """Known spectrum of Q = Gamma5 D (n = 48): from random starts the refined
    block reaches eigen-residual 1e-10 with Ritz values equal to the four
    eigenvalues of smallest modulus (in that order) and vectors equal to the
    eigenvectors up to the fixed phase (sum of entries real, positive)."""
    W, lam, Dm = _known_spectrum()
    Dinv = np.linalg.inv(Dm)
    rng = np.random.default_rng(4)
    V0 = rng.standard_normal((48, 4)) + 1j * rng.standard_normal((48, 4))
    V, rho, steps = refine_test_vectors(lambda v: Dm @ v, lambda b: Dinv @ b, V0, 200, 1e-10)
    assert rho.max() <= 1e-10 and 0 < steps < 200
    for i in range(4):
        w = W[:, i] * np.conj(W[:, i].sum()) / abs(W[:, i].sum())
        assert np.linalg.norm(V[:, i] - w) < 1e-9, i
        assert abs(np.sum(V[:, i]).imag) < 1e-12 and np.sum(V[:, i]).real > 0


def test_refine_eigen_residual_by_hand():
    """One column v = (w1 + eps w2)/sqrt(1 + eps^2) of two eigenvectors: no
    power step (max_iters 0) returns theta = (l1 + eps^2 l2)/(1 + eps^2) and
    rho = sqrt((l1 - theta)^2 + eps^2 (l2 - theta)^2) / (sqrt(1 + eps^2) |theta|)."""
    W, lam, Dm = _known_spectrum()
    eps = 0.1
    v = (W[:, 0] + eps * W[:, 5]) / np.sqrt(1 + eps ** 2)
    V, rho, steps = refine_test_vectors(lambda x: Dm @ x, None, v[:, None], 0, 0.0)
    l1, l2 = lam[0], lam[5]
    th = (l1 + eps ** 2 * l2) / (1 + eps ** 2)
    want = np.sqrt((l1 - th) ** 2 + eps ** 2 * (l2 - th) ** 2) / (np.sqrt(1 + eps ** 2) * abs(th))
    assert steps == 0 and abs(rho[0] - want) < 1e-13 * want
    # exact eigenvectors have zero residual
    V, rho, steps = refine_test_vectors(lambda x: Dm @ x, None, W[:, :3].copy(), 0, 0.0)
    assert rho.max() < 1e-12
