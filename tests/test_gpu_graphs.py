"""Form (2) machinery: captured coarse-grid corrections replayed from HIP
graphs, and the launch-shape autotuner.

Graph replays run the same kernels with the same arguments as the eager
path and every reduction sums in a fixed order, so the results must be
bitwise identical, replay after replay, with eager work and synchronisation
between the replays.  Autotuned variants change only the launch shape (and,
for the rhs-per-thread choice, FP32 rounding order): within 1e-6 of the
untuned FP32 result.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from gpu_common import to_gpu, from_gpu, rel  # noqa: E402
from lattice_inputs import gauge_field, random_spinor  # noqa: E402


@pytest.fixture(scope="module")
def side():
    import torch
    import paper_2509_11424_amd as m

    class P:
        pass

    p = P()
    p.stream = torch.cuda.Stream(device=0)  # graphs need a non-default stream
    p.ctx = m.Context(0, stream=p.stream.cuda_stream)
    p.U = gauge_field((4, 4, 4, 8), 0.6, 71)
    p.op = m.Operator(p.ctx, p.U, 0.05, 1.0)
    p.h = m.Hierarchy(p.op, [(2, 2, 2, 2), (1, 1, 1, 2)], [8, 8], seed=72, max_nrhs=8, restart=16, mixed=1)
    torch.cuda.synchronize()
    return p


def _b(V, nrhs, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((nrhs, V, 12)) + 1j * rng.standard_normal((nrhs, V, 12))


def test_graph_replays_match_eager_bitwise(side):
    import torch
    import paper_2509_11424_amd as m
    p = side
    V = p.op.V
    b = to_gpu(_b(V, 6, 73))
    torch.cuda.synchronize()
    eager = m.solve_desc(tol=1e-10, kind="mg_mixed", smooth=3, coarse_iters=4, maxiter=3000, graphs=False)
    graph = m.solve_desc(tol=1e-10, kind="mg_mixed", smooth=3, coarse_iters=4, maxiter=3000, graphs=True)
    x0, st0 = p.h.solve(0, b, eager)  # returns after the library's stream finished
    x0 = x0.clone()
    y = torch.empty_like(b)
    for rep in range(4):  # first use eager, second captures, then replays
        x, st = p.h.solve(0, b, graph)
        assert torch.equal(x, x0), rep
        assert st["iterations"] == st0["iterations"]
        p.op.apply(b, y)  # eager work on the same stream between replays
        p.stream.synchronize()
    assert st["max_rel_residual"] <= 1e-10


def test_graph_estimates_match_eager(side):
    import paper_2509_11424_amd as m
    p = side
    eager = m.solve_desc(tol=1e-10, kind="mg_mixed", smooth=2, coarse_iters=3, maxiter=3000, graphs=False)
    graph = m.solve_desc(tol=1e-10, kind="mg_mixed", smooth=2, coarse_iters=3, maxiter=3000, graphs=True)
    a = p.h.estimate("trace", "orthogonal", [4, 8, 8], seed=74, batch=[4, 8, 8], solve=eager)
    for _ in range(2):
        g = p.h.estimate("trace", "orthogonal", [4, 8, 8], seed=74, batch=[4, 8, 8], solve=graph)
        for sa, sg in zip(a["samples"], g["samples"]):
            assert np.array_equal(sa, sg)


def test_autotuner_keeps_results(side):
    import torch
    import paper_2509_11424_amd as m
    p = side
    dims = (4, 4, 4, 8)
    x = to_gpu(random_spinor(dims, 75, batch=8).reshape(8, -1, 12)).to(torch.complex64)
    torch.cuda.synchronize()
    y0 = p.op.apply(x, prec="f32")
    p.stream.synchronize()  # the library runs on the side stream, torch on the default one
    p.ctx.autotune(True)
    try:
        y1 = p.op.apply(x, prec="f32")
        y2 = p.op.apply(x, prec="f32")  # tuned shape reused
        p.stream.synchronize()
        s = m.solve_desc(tol=1e-10, kind="mg_mixed", maxiter=3000)
        bb = to_gpu(_b(p.op.V, 8, 76))
        torch.cuda.synchronize()
        xs, st = p.h.solve(0, bb, s)
    finally:
        p.ctx.autotune(False)
    p.stream.synchronize()
    assert rel(from_gpu(y1.to(torch.complex128)), from_gpu(y0.to(torch.complex128))) < 1e-6
    assert torch.equal(y1, y2)
    rep = p.ctx.tune_report()
    keys = [k for k in rep if k.startswith("dslash/1/")]
    assert keys, rep
    for k, (v, ms) in rep.items():
        assert 0 <= v < len(ms) and all(t > 0 for t in ms)
    # the FP32 dslash at 8 rhs has four shapes (rhs per thread x block order)
    assert len(rep[keys[0]][1]) == 4
    assert st["max_rel_residual"] <= 1e-10
