"""Pins of the oracle's estimators: exact traces, telescoping, unbiasedness,
variance identity, correlator and loop decompositions, MLMC allocation."""
import numpy as np
import pytest

from lattice_inputs import gauge_field
from oracle.dirac import WilsonClover, gamma5
from oracle.multigrid import Hierarchy
from oracle.solve import level_solver
from oracle.philox import z4_vector, stream_id, KIND_O, KIND_CORR, KIND_LOOP
from oracle import estimators as E


@pytest.fixture(scope="module")
def setup():
    U = gauge_field((4, 4, 4, 4), 0.5, 12)
    D = WilsonClover(U, 0.05, 1.0)
    h = Hierarchy(D, [(2, 2, 2, 2)], [8], seed=102)
    solvers = [level_solver(op) for op in h.ops]
    ex = E.exact_operators(h)
    return h, solvers, ex


def test_telescoping_identities(setup):
    h, _, ex = setup
    t0 = np.trace(ex["Dinv"][0])
    tc = np.trace(ex["Dinv"][1])
    assert abs(np.trace(ex["O"][0]) + np.trace(ex["F"][0]) + tc - t0) < 1e-12 * abs(t0)
    assert abs(np.trace(ex["M"][0]) + tc - t0) < 1e-12 * abs(t0)
    # two-sided projection leaves the trace unchanged (Sec. 3)
    P = ex["P"][0]
    Q = np.eye(P.shape[0]) - P @ P.conj().T
    assert abs(np.trace(Q @ ex["Dinv"][0]) - np.trace(ex["O"][0])) < 1e-12 * abs(t0)
    # orthogonal projector does not increase the Frobenius norm (Sec. 3)
    assert np.linalg.norm(Q @ ex["Dinv"][0]) <= np.linalg.norm(ex["Dinv"][0])


def test_per_probe_values_match_dense_quadratic_forms(setup):
    h, solvers, ex = setup
    seed = 55
    X = E.O_samples(h, solvers, 0, seed, 3)
    for k in range(3):
        x = z4_vector(h.ops[0].n, seed, stream_id(0, KIND_O), k)
        assert abs(X[k] - np.vdot(x, ex["O"][0] @ x)) < 1e-10 * abs(X[k])
    XF = E.F_samples(h, solvers, 0, seed, 3)
    XM = E.M_samples(h, solvers, 0, seed, 3)
    XC = E.coarsest_samples(h, solvers, seed, 3)
    XP = E.plain_samples(h, solvers, seed, 3)
    from oracle.philox import KIND_F, KIND_M, KIND_COARSEST, KIND_PLAIN
    for k in range(3):
        x = z4_vector(h.ops[1].n, seed, stream_id(0, KIND_F), k)
        assert abs(XF[k] - np.vdot(x, ex["F"][0] @ x)) < 1e-9 * max(1, abs(XF[k]))
        x = z4_vector(h.ops[0].n, seed, stream_id(0, KIND_M), k)
        assert abs(XM[k] - np.vdot(x, ex["M"][0] @ x)) < 1e-10 * abs(XM[k])
        x = z4_vector(h.ops[1].n, seed, stream_id(1, KIND_COARSEST), k)
        assert abs(XC[k] - np.vdot(x, ex["Dinv"][1] @ x)) < 1e-10 * abs(XC[k])
        x = z4_vector(h.ops[0].n, seed, stream_id(0, KIND_PLAIN), k)
        assert abs(XP[k] - np.vdot(x, ex["Dinv"][0] @ x)) < 1e-10 * abs(XP[k])


def test_unbiased_within_error_bars(setup):
    h, solvers, ex = setup
    N = 64
    for name, fn, A in [("O", lambda: E.O_samples(h, solvers, 0, 9, N), ex["O"][0]),
                        ("F", lambda: E.F_samples(h, solvers, 0, 9, N), ex["F"][0]),
                        ("c", lambda: E.coarsest_samples(h, solvers, 9, N), ex["Dinv"][1])]:
        X = fn()
        sigma = np.sqrt(E.offdiag_fro2(A) / N)
        assert abs(X.mean() - np.trace(A)) < 5 * sigma, name
        # sample variance within a generous band of the exact Z4 variance
        _, v = E.mean_var(X)
        assert 0.4 < v / E.offdiag_fro2(A) < 2.0, name


def test_variance_ordering_trend(setup):
    """Orthogonal terms have smaller Z4 variance than plain and oblique ones
    (trend reported in Sec. 4.2; on this lattice it holds exactly)."""
    _, _, ex = setup
    v_plain = E.offdiag_fro2(ex["Dinv"][0])
    v_O = E.offdiag_fro2(ex["O"][0])
    v_F = E.offdiag_fro2(ex["F"][0])
    v_M = E.offdiag_fro2(ex["M"][0])
    assert v_O < v_plain and v_O < v_M and v_F < 0.1 * v_O


@pytest.mark.parametrize("dec", ["plain", "oblique", "orthogonal"])
def test_exact_correlator_decomposition_sums_to_plain(setup, dec):
    h, _, _ = setup
    Gp, _ = E.exact_correlator(h, "plain")
    G, _ = E.exact_correlator(h, dec)
    np.testing.assert_allclose(G.sum(axis=(0, 1)), Gp[0, 0], rtol=1e-11)
    # plain correlator: G(t) = (1/T) sum_t' ||D^-1(t+t',t')||_F^2 (real, > 0)
    assert np.all(Gp[0, 0].real > 0) and np.abs(Gp[0, 0].imag).max() < 1e-12 * Gp[0, 0].real.max()


def test_correlator_per_probe_matches_dense_terms(setup):
    """Per-probe X_rs(t) from solves equals the one-end estimator built from
    the dense B_r and B~_s = G5 B_s^H G5 for the same source."""
    h, solvers, _ = setup
    G, Bs = E.exact_correlator(h, "orthogonal")
    pairs, X = E.correlator_samples(h, solvers, "orthogonal", 0, seed=77, nprobe=1)
    dims = h.ops[0].dims
    T = dims[3]
    n = h.ops[0].n
    g5 = np.tile(np.repeat(np.diag(gamma5()).real, 3), h.ops[0].V)
    eta = z4_vector(n, 77, stream_id(0, KIND_CORR), 0)
    sl = np.repeat(np.arange(T), dims[0] * dims[1] * dims[2] * 12)
    for ip, (r, s) in enumerate(pairs):
        Bt = g5[:, None] * Bs[s].conj().T * g5[None, :]
        want = np.zeros(T, dtype=complex)
        for tp in range(T):
            e = np.where(sl == tp, eta, 0)
            a, b = Bs[r] @ e, Bt @ e
            for t in range(T):
                m = sl == (t + tp) % T
                want[t] += np.vdot(b[m], a[m]) / T
        np.testing.assert_allclose(X[0, ip], want, rtol=1e-9, atol=1e-12 * np.abs(want).max())


def test_correlator_groups_cover_all_pairs(setup):
    h, solvers, _ = setup
    lv = E.term_levels(h.L, "orthogonal")
    R = len(lv)
    seen = []
    for g in range(h.L):
        pairs = [(r, s) for r in range(R) for s in range(R) if min(lv[r], lv[s]) == g]
        seen += pairs
    assert sorted(seen) == [(r, s) for r in range(R) for s in range(R)]


@pytest.mark.parametrize("dec", ["oblique", "orthogonal"])
def test_loop_terms_sum_to_plain_per_probe(setup, dec):
    """sum_r B_r = D^-1, so with the same eta the per-probe loop values of all
    terms add up to the plain one (eq. trace_equality_disconnected)."""
    h, solvers, _ = setup
    lv = E.term_levels(h.L, dec)
    ops = E.TermOperators(h, solvers, dec)
    opp = E.TermOperators(h, solvers, "plain")
    eta = z4_vector(h.ops[0].n, 3, stream_id(0, KIND_LOOP), 0)
    tot = sum(ops.apply(r, eta, False) for r in range(len(lv)))
    np.testing.assert_allclose(tot, opp.apply(0, eta, False), atol=1e-10)


def test_loop_estimator_unbiased(setup):
    h, solvers, ex = setup
    terms, X = E.loop_samples(h, solvers, "plain", 0, seed=5, nprobe=24)
    Dinv = ex["Dinv"][0]
    dims = h.ops[0].dims
    T = dims[3]
    per = dims[0] * dims[1] * dims[2] * 12
    G = E.gamma_list()
    for ig in (0, 1):
        for t in (0, 2):
            idx = slice(t * per, (t + 1) * per)
            Gam = np.kron(np.eye(per // 12), np.kron(G[ig], np.eye(3)))
            A_full = np.zeros_like(Dinv)
            A_full[idx, :] = Gam @ Dinv[idx, :]
            exact = np.trace(A_full)
            sigma = np.sqrt(E.offdiag_fro2(A_full) / 24)
            assert abs(X[:, 0, ig, t].mean() - exact) < 5 * sigma


def test_mlmc_allocation_closed_form():
    V = np.array([4.0, 1.0, 0.25])
    C = np.array([1.0, 8.0, 64.0])
    eps2 = 1e-3
    N = E.mlmc_allocation(V, C, eps2)
    assert abs(np.sum(V / N) - eps2) < 1e-15
    assert abs(np.sum(N * C) - np.sum(np.sqrt(V * C)) ** 2 / eps2) < 1e-8


def _slice_index(dims):
    return np.repeat(np.arange(dims[3]), dims[0] * dims[1] * dims[2] * 12)


def test_plain_correlator_is_frobenius_norm_of_slice_blocks(setup):
    """Sec. 1.1, eq. connected-G with Gamma5-hermiticity D^-1(t',t1) =
    G5 D^-1(t1,t')^H G5: G(t) = (1/T) sum_t' ||D^-1(t+t', t')||_F^2, computed
    here straight from the dense inverse (no Gamma5 algebra).  A slip in the
    Gamma5 placement or in the slice pairing of exact_correlator breaks it."""
    h, _, ex = setup
    Dinv = ex["Dinv"][0]
    dims = h.ops[0].dims
    T = dims[3]
    sl = _slice_index(dims)
    want = np.zeros(T)
    for t in range(T):
        for tp in range(T):
            blk = Dinv[np.ix_(sl == (t + tp) % T, sl == tp)]
            want[t] += np.sum(np.abs(blk) ** 2) / T
    G, _ = E.exact_correlator(h, "plain")
    np.testing.assert_allclose(G[0, 0].real, want, rtol=1e-12)
    assert np.abs(G[0, 0].imag).max() < 1e-12 * want.max()
    # ||D^-1(a, b)||_F = ||D^-1(b, a)||_F by Gamma5-hermiticity, so G(t) = G(-t)
    np.testing.assert_allclose(want, np.roll(want[::-1], 1), rtol=1e-12)
    # and the pairing of slices is not the trivial one: G(0) differs from G(1)
    assert abs(want[0] - want[1]) > 1e-3 * want[0]


def test_plain_correlator_samples_unbiased_with_exact_variance(setup):
    """The plain one-end estimator of one probe is the real quadratic form
    X(t) = eta^H A_t eta with A_t = (1/T) blockdiag_t'(D^-1(t+t',t')^H
    D^-1(t+t',t')): its mean is G(t) above and its Z4 variance is
    ||offdiag(A_t)||_F^2 (eq. variance-Frobenius-Relation).  The sample mean of
    N probes lies within 5 sigma of the Frobenius-norm value."""
    h, solvers, ex = setup
    Dinv = ex["Dinv"][0]
    dims = h.ops[0].dims
    T = dims[3]
    sl = _slice_index(dims)
    N = 24
    _, X = E.correlator_samples(h, solvers, "plain", 0, seed=31, nprobe=N)
    assert np.abs(X.imag).max() < 1e-12 * np.abs(X.real).max()
    for t in range(T):
        A = np.zeros_like(Dinv)
        for tp in range(T):
            m1, m0 = sl == (t + tp) % T, sl == tp
            blk = Dinv[np.ix_(m1, m0)]
            A[np.ix_(m0, m0)] += blk.conj().T @ blk / T
        sigma = np.sqrt(E.offdiag_fro2(A) / N)
        assert abs(X[:, 0, t].mean() - np.trace(A)) < 5 * sigma, t


def test_loop_probing_unbiased_with_exact_coloured_variance(setup):
    """Probing sources (2^4 colours, oracle/noise.py) for the loop
    tr(Gamma5 D^-1(t, t)): the coloured estimator is unbiased, its Z4 variance
    is the sum of |A_ij|^2 over i != j of equal colour, and on this field it
    is below the plain Z4 variance ||offdiag A||_F^2 (Sec. 5, probing)."""
    from oracle.noise import site_colours
    h, solvers, ex = setup
    Dinv = ex["Dinv"][0]
    dims = h.ops[0].dims
    per = dims[0] * dims[1] * dims[2] * 12
    G = E.gamma_list()
    t, ig = 1, 1
    idx = slice(t * per, (t + 1) * per)
    A = np.zeros_like(Dinv)
    A[idx, :] = np.kron(np.eye(per // 12), np.kron(G[ig], np.eye(3))) @ Dinv[idx, :]
    col = np.repeat(site_colours(dims, 2), 12)
    same = col[:, None] == col[None, :]
    v_col = float(np.sum(np.abs(A[same]) ** 2) - np.sum(np.abs(np.diag(A)) ** 2))
    v_plain = E.offdiag_fro2(A)
    assert v_col < 0.5 * v_plain
    N = 12
    _, X = E.loop_samples(h, solvers, "plain", 0, seed=8, nprobe=N, probing=2)
    assert abs(X[:, 0, ig, t].mean() - np.trace(A)) < 5 * np.sqrt(v_col / N)
    # probing distance 1 is plain
    _, X1 = E.loop_samples(h, solvers, "plain", 0, seed=8, nprobe=2, probing=1)
    _, X0 = E.loop_samples(h, solvers, "plain", 0, seed=8, nprobe=2)
    np.testing.assert_allclose(X1, X0, rtol=0, atol=0)
