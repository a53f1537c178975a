"""Mixed-precision form: FP32/FP16 fine dslash, FP32/BF16 MFMA coarse stencils,
FP64 defect correction.  Parity against the FP64 oracle.

Bars: FP64 MFMA coarse stencil 1e-13 (rounding order only); FP32 coarse
stencil 2e-6 (u = 6e-8 times the 9 d-term dot products); BF16 coarse stencil
2e-2 (operands rounded to BF16, u = 3.9e-3, accumulated in FP32); solutions
of the mixed solver at tol 1e-12 within 1e-9 of the oracle's dense solve;
per-probe quadratic forms within 1e-8 relative.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from gpu_common import to_gpu, from_gpu, rel  # noqa: E402
from lattice_inputs import gauge_field  # noqa: E402


@pytest.fixture(scope="module")
def three():
    import paper_2509_11424_amd as m
    from oracle.dirac import WilsonClover
    from oracle.multigrid import Hierarchy
    from oracle.solve import level_solver

    class P:
        pass

    p = P()
    ctx = m.Context(0)
    p.ctx = ctx
    p.U = gauge_field((4, 4, 4, 8), 0.6, 31)
    p.op = m.Operator(ctx, p.U, 0.05, 1.0)
    p.h = m.Hierarchy(p.op, [(2, 2, 2, 2), (1, 1, 1, 2)], [8, 8], seed=17, max_nrhs=8, restart=20, mixed=2)
    p.D = WilsonClover(p.U, 0.05, 1.0)
    p.oh = Hierarchy(p.D, [(2, 2, 2, 2), (1, 1, 1, 2)], [8, 8], seed=17)
    p.solvers = [level_solver(o) for o in p.oh.ops]
    return p


def _rand(s, d, nrhs, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((nrhs, s, d)) + 1j * rng.standard_normal((nrhs, s, d))


@pytest.mark.parametrize("prec,bound", [("f64", 1e-13), ("f32", 2e-6), ("bf16", 2e-2)])
def test_coarse_stencil_precisions(three, prec, bound):
    import torch
    p = three
    for l in (1, 2):
        s, d, n = p.h.level_info(l)
        x = _rand(s, d, 5, l)
        want = p.oh.ops[l].matvec(x.reshape(5, -1))
        xg = to_gpu(x)
        if prec != "f64":
            xg = xg.to(torch.complex64)
        y = p.h.apply_prec(l, xg, prec).to(torch.complex128)
        assert rel(from_gpu(y).reshape(5, -1), want) < bound, (l, prec)


def test_coarse_bf16_launch_shapes_agree(three):
    """Every launch shape of the BF16 MFMA stencil (waves per workgroup, 16-rhs
    tiles per wave) on a ragged rhs count (70 = 4 x 16 + 6): each tile runs the
    same MFMA sequence in every shape, so the results are bitwise equal; all
    within the BF16 bound of the oracle."""
    import torch
    p = three
    nrhs = 70
    for l in (1, 2):
        s, d, n = p.h.level_info(l)
        x = _rand(s, d, nrhs, 10 + l)
        want = p.oh.ops[l].matvec(x.reshape(nrhs, -1))
        xg = to_gpu(x).to(torch.complex64)
        key = "coarsebf16/%d/%d/%d" % (s, d, nrhs)
        p.ctx.autotune(True)
        try:
            p.h.apply_prec(l, xg, "bf16")
        finally:
            p.ctx.autotune(False)
        torch.cuda.synchronize()
        nvar = len(p.ctx.tune_report()[key][1])
        assert nvar >= 5  # three workgroup sizes, then two and four tiles per wave
        p.ctx.tune_set(key, 0)
        y0 = p.h.apply_prec(l, xg, "bf16")
        for v in range(1, nvar):
            p.ctx.tune_set(key, v)
            y = p.h.apply_prec(l, xg, "bf16")
            torch.cuda.synchronize()
            assert torch.equal(y, y0), (l, v)
        p.ctx.tune_set(key, 0)
        assert rel(from_gpu(y0.to(torch.complex128)).reshape(nrhs, -1), want) < 2e-2


def test_fine_operator_f16_through_hierarchy(three):
    import torch
    p = three
    s, d, n = p.h.level_info(0)
    x = _rand(s, d, 2, 3)
    want = p.D.matvec(x.reshape(2, -1))
    xh = torch.view_as_real(to_gpu(x)).to(torch.float16).contiguous()
    y = p.h.apply_prec(0, xh, "f16")
    y = torch.view_as_complex(y.float().contiguous()).to(torch.complex128)
    assert rel(from_gpu(y).reshape(2, -1), want) < 4e-3


@pytest.mark.parametrize("bf16", [False, True])
def test_mixed_solves_reach_fp64_accuracy(three, bf16):
    import paper_2509_11424_amd as m
    p = three
    for l in range(3):
        s, d, n = p.h.level_info(l)
        b = _rand(s, d, 4, 40 + l)
        sd = m.solve_desc(tol=1e-12, kind="mg_mixed", coarse_bf16=bf16, maxiter=4000)
        x, st = p.h.solve(l, to_gpu(b), sd)
        assert st["max_rel_residual"] <= 1e-12
        want = np.stack([p.solvers[l](bb) for bb in b.reshape(4, -1)])
        assert rel(from_gpu(x).reshape(4, -1), want) < 1e-9


def test_mixed_estimate_per_probe(three):
    import paper_2509_11424_amd as m
    from oracle import estimators as E
    p = three
    sd = m.solve_desc(tol=1e-12, kind="mg_mixed", coarse_bf16=True, maxiter=4000)
    res = p.h.estimate("trace", "orthogonal", [3, 3, 3], seed=61, batch=3, solve=sd)
    want = [E.O_samples(p.oh, p.solvers, l, 61, 3) for l in range(2)]
    want += [E.F_samples(p.oh, p.solvers, l, 61, 3) for l in range(2)]
    want += [E.coarsest_samples(p.oh, p.solvers, 61, 3)]
    scale0 = np.abs(E.plain_samples(p.oh, p.solvers, 61, 1)[0])
    for q in range(5):
        got = res["samples"][q][:, 0, 0]
        assert np.all(np.abs(got - want[q]) <= 1e-8 * (np.abs(want[q]) + scale0)), q
