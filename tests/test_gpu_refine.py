"""GPU parity of the test-vector refinement (Sec. 5: test vectors of smaller
eigen-residual; reading in oracle/multigrid.py, refine_test_vectors) against
the FP64 oracle on a 4^4 clover lattice, 2^4 aggregates, N_tv 8.

Three inverse block power steps with Rayleigh-Ritz (eig_tol 0 forces the
step count), solves to 1e-12 on the GPU and a dense LU in the oracle.  Bars:
Ritz values within 1e-10 and eigen-residuals within 1e-8 (relative), the
rebuilt P and D_c within 1e-9, per-probe orthogonal tr(D^-1) values within
1e-8 of |a| + |b|.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from gpu_common import rel  # noqa: E402
from lattice_inputs import gauge_field  # noqa: E402


def test_refined_hierarchy_matches_oracle():
    import paper_2509_11424_amd as m
    from oracle.dirac import WilsonClover
    from oracle.multigrid import Hierarchy
    from oracle.solve import level_solver
    from oracle import estimators as E
    ctx = m.Context(0)
    U = gauge_field((4, 4, 4, 4), 0.5, 12)
    op = m.Operator(ctx, U, 0.05, 1.0)
    h = m.Hierarchy(op, [(2, 2, 2, 2)], [8], seed=102, max_nrhs=4, restart=20, mixed=2)
    st = h.refine(max_iters=3, eig_tol=0.0, power_tol=1e-12, batch=3, solve=m.solve_desc(tol=1e-12))
    assert st["steps"] == 3 and st["converged"]
    D = WilsonClover(U, 0.05, 1.0)
    Dinv = np.linalg.inv(D.dense())
    oh = Hierarchy(D, [(2, 2, 2, 2)], [8], seed=102, refine=(lambda b: Dinv @ b, 3, 0.0))
    assert oh.refine_steps == 3
    np.testing.assert_allclose(st["rho"], oh.refine_rho, rtol=1e-8)
    assert st["max_rho"] > 0 and st["max_rho_start"] > 0
    assert rel(h.export(0, "P"), oh.transfers[0].P) < 1e-9
    assert rel(h.export(0, "coarse"), oh.ops[1].blocks) < 1e-9
    solvers = [level_solver(o) for o in oh.ops]
    res = h.estimate("trace", "orthogonal", [3, 3], seed=29, batch=3, solve=m.solve_desc(tol=1e-12))
    want = [E.O_samples(oh, solvers, 0, 29, 3), E.F_samples(oh, solvers, 0, 29, 3),
            E.coarsest_samples(oh, solvers, 29, 3)]
    sc = np.abs(E.plain_samples(oh, solvers, 29, 1)[0])
    for q in range(3):
        got = res["samples"][q][:, 0, 0]
        assert np.all(np.abs(got - want[q]) <= 1e-8 * (np.abs(want[q]) + sc)), q
    # the mixed solver runs on the rebuilt operators
    r2 = h.estimate("trace", "orthogonal", [3, 3], seed=29, batch=3,
                    solve=m.solve_desc(tol=1e-12, kind="mg_mixed", maxiter=4000))
    for q in range(3):
        got = r2["samples"][q][:, 0, 0]
        assert np.all(np.abs(got - want[q]) <= 1e-8 * (np.abs(want[q]) + sc)), q
