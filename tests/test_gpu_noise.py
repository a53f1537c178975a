"""GPU parity of the probe distributions (Sec. 1: Z4, Z2, U(1), real
Gaussian) and of probing sources for loops (Sec. 5) against the oracle
(oracle/noise.py, oracle/estimators.py).

Bars: Z4 and Z2 entries bit-exact (integer decisions of the Philox words);
U(1) and Gaussian entries within 1e-14 (FP64 cos / sin / log of the device
library against numpy's); per-probe estimator values within 1e-8 relative
(differences X = a - b against |a| + |b| through the plain value's scale).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from lattice_inputs import gauge_field  # noqa: E402


@pytest.fixture(scope="module")
def nz():
    import paper_2509_11424_amd as m
    from oracle.dirac import WilsonClover
    from oracle.multigrid import Hierarchy
    from oracle.solve import level_solver

    class P:
        pass

    p = P()
    p.ctx = m.Context(0)
    p.U = gauge_field((4, 4, 4, 4), 0.5, 12)
    p.op = m.Operator(p.ctx, p.U, 0.05, 1.0)
    p.h = m.Hierarchy(p.op, [(2, 2, 2, 2)], [8], seed=102, max_nrhs=4, restart=20, with_corr=True)
    D = WilsonClover(p.U, 0.05, 1.0)
    p.oh = Hierarchy(D, [(2, 2, 2, 2)], [8], seed=102)
    p.solvers = [level_solver(o) for o in p.oh.ops]
    return p


@pytest.mark.parametrize("kind", ["z4", "z2", "u1", "gauss"])
def test_draws_match_oracle(nz, kind):
    import paper_2509_11424_amd as m
    from oracle.noise import noise_vector, NOISE_NAMES
    nsite, dof, nprobe = 300, 12, 3
    for prec in ("f64", "f32"):
        x = m.draw_noise(nz.ctx, kind, 77, 513, 5, nprobe, nsite, dof, prec).cpu().numpy()
        for p in range(nprobe):
            want = noise_vector(nsite * dof, 77, 513, 5 + p, NOISE_NAMES[kind])
            got = x[:, :, p].T.reshape(-1)  # entry index site * dof + dof_index
            if kind in ("z4", "z2"):
                assert np.array_equal(got, want.astype(got.dtype)), (kind, prec, p)
            else:
                tol = 1e-14 if prec == "f64" else 1e-6
                assert np.abs(got - want).max() <= tol * max(1.0, np.abs(want).max()), (kind, prec, p)


@pytest.mark.parametrize("kind", ["z2", "u1", "gauss"])
def test_orthogonal_trace_with_other_noise(nz, kind):
    import paper_2509_11424_amd as m
    from oracle import estimators as E
    from oracle.noise import NOISE_NAMES
    p = nz
    k = NOISE_NAMES[kind]
    res = p.h.estimate("trace", "orthogonal", [3, 3], seed=19, batch=3, solve=m.solve_desc(tol=1e-12), noise=kind)
    want = [E.O_samples(p.oh, p.solvers, 0, 19, 3, noise=k), E.F_samples(p.oh, p.solvers, 0, 19, 3, noise=k),
            E.coarsest_samples(p.oh, p.solvers, 19, 3, noise=k)]
    scale = np.abs(E.plain_samples(p.oh, p.solvers, 19, 1, noise=k)[0])
    for q in range(3):
        got = res["samples"][q][:, 0, 0]
        assert np.all(np.abs(got - want[q]) <= 1e-8 * (np.abs(want[q]) + scale)), (kind, q)


@pytest.mark.parametrize("dec", ["plain", "orthogonal"])
def test_loops_with_probing(nz, dec):
    """Loops with 2^4-coloured probing sources (16 colours, each a solve per
    term) against the oracle, per probe, term, Gamma and t."""
    import paper_2509_11424_amd as m
    from oracle import estimators as E
    p = nz
    L = p.oh.L
    res = p.h.estimate("loops", dec, [2] * L, seed=23, batch=2, solve=m.solve_desc(tol=1e-12), probing=2)
    groups = [0] if dec == "plain" else range(L)
    for g in groups:
        terms, X = E.loop_samples(p.oh, p.solvers, dec, g, seed=23, nprobe=2, probing=2)
        for it, r in enumerate(terms):
            got = res["samples"][r]
            scale = np.abs(X[:, it]).max()
            assert np.abs(got - X[:, it]).max() <= 1e-8 * scale, (dec, g, r)


def test_probing_argument_checks(nz):
    import paper_2509_11424_amd as m
    p = nz
    sd = m.solve_desc(tol=1e-10)
    with pytest.raises(m.MgmError, match="INVALID_ARG"):
        p.h.estimate("trace", "plain", [2, 0], seed=1, batch=2, solve=sd, probing=2)
    with pytest.raises(m.MgmError, match="SHAPE"):
        p.h.estimate("loops", "plain", [2, 0], seed=1, batch=2, solve=sd, probing=3)
    with pytest.raises(m.MgmError, match="INVALID_ARG"):
        p.h.estimate("trace", "plain", [2, 0], seed=1, batch=2, solve=sd, noise=7)
