"""Hierarchies with more test vectors (Sec. 5: N_tv beyond the 24-32 of the
production settings, up to 64 and 128), against the FP64 oracle.

deep: 4 x 4 x 4 x 8 clover lattice, aggregates 2^4 then (1, 1, 1, 2),
N_tv 64 then 8: the first coarse level has 128 dof per site (eight 16-row
MFMA tiles), transfers carry 64 test vectors (the FP64 prolongation splits
its rhs into tiles of 32) and the fine Galerkin product runs in four column
chunks; the second Galerkin product stages 128-dof rows.
wide: 8^4, aggregates 2^4 twice, N_tv 8 then 40: the second coarse level has
80 dof (five MFMA tiles) and its Galerkin product runs in two column chunks.
The refinement of 64 test vectors (block products and CholeskyQR of 64
columns) runs on 4^4.  widest: 128 test vectors, a 256-dof coarse level.

Bars as for the smaller hierarchies: aggregation maps bit-exact; P and D_c
within 1e-10; transfers within 1e-10 (FP64) and 1e-5 (FP32 with FP16 P,
against the oracle's P rounded the same way); the BF16 coarse stencil within
5e-5 of an FP64 stencil built from BF16-rounded blocks; solutions of every
level at tol 1e-12 within 1e-9 of the oracle's; per-probe orthogonal
tr(D^-1) terms within 1e-8 of |a| + |b| (Sec. 3).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from gpu_common import to_gpu, from_gpu, rel  # noqa: E402
from lattice_inputs import gauge_field  # noqa: E402


class _Pair:
    def __init__(self, dims, eps, gseed, m0, blocks, ntv, seed, max_nrhs):
        import paper_2509_11424_amd as m
        from oracle.dirac import WilsonClover
        from oracle.multigrid import Hierarchy
        from oracle.solve import level_solver
        self.ctx = m.Context(0)
        self.U = gauge_field(dims, eps, gseed)
        self.op = m.Operator(self.ctx, self.U, m0, 1.0)
        self.h = m.Hierarchy(self.op, blocks, ntv, seed=seed, max_nrhs=max_nrhs, restart=20, mixed=2)
        D = WilsonClover(self.U, m0, 1.0)
        self.oh = Hierarchy(D, blocks, ntv, seed=seed)
        self.solvers = [level_solver(o) for o in self.oh.ops]


@pytest.fixture(scope="module")
def deep():
    return _Pair((4, 4, 4, 8), 0.5, 64, 0.1, [(2, 2, 2, 2), (1, 1, 1, 2)], [64, 8], 65, max_nrhs=72)


@pytest.fixture(scope="module")
def wide():
    return _Pair((8, 8, 8, 8), 0.5, 66, 0.1, [(2, 2, 2, 2), (2, 2, 2, 2)], [8, 40], 67, max_nrhs=8)


def _rand(sites, dof, nrhs, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((nrhs, sites, dof)) + 1j * rng.standard_normal((nrhs, sites, dof))


def _pairs(deep, wide):
    return {"deep": deep, "wide": wide}


@pytest.mark.parametrize("which", ["deep", "wide"])
def test_maps_P_and_coarse_operators(deep, wide, which):
    p = _pairs(deep, wide)[which]
    for l in range(p.oh.L - 1):
        assert np.array_equal(p.h.export(l, "agg_map"), p.oh.transfers[l].agg.block_index()), (which, l)
        assert rel(p.h.export(l, "P"), p.oh.transfers[l].P) < 1e-10, (which, l)
        assert rel(p.h.export(l, "coarse"), p.oh.ops[l + 1].blocks) < 1e-10, (which, l)
    assert [p.h.level_info(l)[1] for l in range(p.oh.L)] == [12] + [2 * n for n in p.h.desc.ntv[:p.oh.L - 1]]


@pytest.mark.parametrize("nrhs", [1, 33, 70])
def test_transfers_64_vectors(deep, nrhs):
    """FP64 transfers of the 64-vector block (prolongation in rhs tiles of 32:
    one, two and three tiles, the last ragged) and the projector."""
    p = deep
    for l in range(p.oh.L - 1):
        s, d, _ = p.h.level_info(l)
        cs, cd, _ = p.h.level_info(l + 1)
        x = _rand(s, d, nrhs, 100 + l)
        xc = _rand(cs, cd, nrhs, 200 + l)
        tr = p.oh.transfers[l]
        xf, xcf = x.reshape(nrhs, -1), xc.reshape(nrhs, -1)
        assert rel(from_gpu(p.h.restrict(l, to_gpu(x))).reshape(nrhs, -1), tr.restrict(xf)) < 1e-10
        assert rel(from_gpu(p.h.prolong(l, to_gpu(xc))).reshape(nrhs, -1), tr.prolong(xcf)) < 1e-10
        assert rel(from_gpu(p.h.project_out(l, to_gpu(x))).reshape(nrhs, -1), tr.project_out(xf)) < 1e-10


@pytest.mark.parametrize("nrhs", [16, 70])
def test_transfers_f32_fp16_P_64_vectors(deep, nrhs):
    import torch
    from oracle.multigrid import Transfer
    p = deep
    tr = p.oh.transfers[0]
    re = tr.P.real.astype(np.float32).astype(np.float16).astype(np.float64)
    im = tr.P.imag.astype(np.float32).astype(np.float16).astype(np.float64)
    t16 = Transfer(tr.agg, re + 1j * im)
    s, d, _ = p.h.level_info(0)
    cs, cd, _ = p.h.level_info(1)
    x = _rand(s, d, nrhs, 300).astype(np.complex64)
    xc = _rand(cs, cd, nrhs, 400).astype(np.complex64)
    yc = p.h.restrict(0, to_gpu(x).to(torch.complex64), prec="f32")
    y = p.h.prolong(0, to_gpu(xc).to(torch.complex64), prec="f32")
    assert rel(from_gpu(yc).reshape(nrhs, -1), t16.restrict(x.astype(np.complex128).reshape(nrhs, -1))) < 1e-5
    assert rel(from_gpu(y).reshape(nrhs, -1), t16.prolong(xc.astype(np.complex128).reshape(nrhs, -1))) < 1e-5


def _bf16(a):
    """round to nearest even BF16 after rounding to FP32 (as the device does)"""
    b = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("which,level", [("deep", 1), ("wide", 2)])
def test_coarse_stencils_wide_blocks(deep, wide, which, level):
    """d = 128 (eight MFMA row tiles) and d = 80 (five, the last partly
    padded): FP64 within 1e-10 of the oracle stencil (the bar of D_c), FP32
    within 2e-6, BF16
    against the stencil of BF16-rounded blocks on BF16-rounded inputs."""
    import torch
    p = _pairs(deep, wide)[which]
    op = p.oh.ops[level]
    B, nbr = op.stencil()
    d, V = op.d, op.V
    nrhs = 21
    x = _rand(V, d, nrhs, 500 + level)
    want = op.matvec(x.reshape(nrhs, -1))
    got = p.h.apply_prec(level, to_gpu(x), "f64")
    assert rel(from_gpu(got).reshape(nrhs, -1), want) < 1e-10  # D_c itself agrees to 1e-10
    x32 = x.astype(np.complex64)
    got = p.h.apply_prec(level, to_gpu(x32), "f32")
    assert rel(from_gpu(got).astype(np.complex128).reshape(nrhs, -1), op.matvec(x32.astype(np.complex128).reshape(nrhs, -1))) < 2e-6
    g = np.where(np.arange(d) < d // 2, 1.0, -1.0)
    Bf = _bf16(B[:, :5].real) + 1j * _bf16(B[:, :5].imag)
    blocks = np.concatenate([Bf] + [
        (g[None, :, None] * np.conj(np.transpose(Bf[nbr[5 + mu], 1 + mu], (0, 2, 1))) * g[None, None, :])[:, None]
        for mu in range(4)], axis=1)
    xr = _bf16(x32.real) + 1j * _bf16(x32.imag)
    want = np.zeros((nrhs, V, d), dtype=np.complex128)
    for k in range(9):
        want += np.einsum("sij,nsj->nsi", blocks[:, k], xr[:, nbr[k], :])
    got = p.h.apply_prec(level, to_gpu(x32), "bf16")
    assert got.dtype == torch.complex64
    assert rel(from_gpu(got).astype(np.complex128).reshape(nrhs, -1), want.reshape(nrhs, -1)) < 5e-5


@pytest.mark.parametrize("kind", ["mg", "mg_mixed"])
def test_solves_every_level(deep, kind):
    import torch
    import paper_2509_11424_amd as m
    p = deep
    for l in range(p.oh.L):
        s, d, _ = p.h.level_info(l)
        b = _rand(s, d, 3, 70 + l)
        torch.cuda.synchronize()
        x, st = p.h.solve(l, to_gpu(b), m.solve_desc(tol=1e-12, kind=kind, maxiter=4000))
        torch.cuda.synchronize()
        assert st["max_rel_residual"] <= 1e-12, (kind, l)
        want = np.stack([p.solvers[l](bb) for bb in b.reshape(3, -1)])
        assert rel(from_gpu(x).reshape(3, -1), want) < 1e-9, (kind, l)


@pytest.mark.parametrize("which", ["deep", "wide"])
def test_orthogonal_trace_per_probe(deep, wide, which):
    import paper_2509_11424_amd as m
    from oracle import estimators as E
    p = _pairs(deep, wide)[which]
    L = p.oh.L
    seed, N = 75, 2
    sd = m.solve_desc(tol=1e-12, kind="mg_mixed", smooth=4, smooth_coarse=2, coarse_iters=2, maxiter=4000,
                      graphs=True)
    res = p.h.estimate("trace", "orthogonal", [N] * L, seed=seed, batch=2, solve=sd)
    want = [E.O_samples(p.oh, p.solvers, l, seed, N) for l in range(L - 1)]
    want += [E.F_samples(p.oh, p.solvers, l, seed, N) for l in range(L - 1)]
    want += [E.coarsest_samples(p.oh, p.solvers, seed, N)]
    sc = np.abs(E.plain_samples(p.oh, p.solvers, seed, 1)[0])
    assert len(res["samples"]) == len(want)
    for q, w in enumerate(want):
        got = res["samples"][q][:, 0, 0]
        assert np.all(np.abs(got - w) <= 1e-8 * (np.abs(w) + sc)), (which, q, got, w)
    assert res["stats"]["max_rel_residual"] <= 1e-12


def test_refined_64_test_vectors():
    """Refinement of 64 test vectors (three inverse block-power steps with
    Rayleigh-Ritz on Gamma5 D, as in tests/test_gpu_refine.py for 8) on a 4^4
    clover lattice with 2^4 aggregates (96 rows per block): eigen-residuals
    within 1e-8 relative, the rebuilt P and D_c within 1e-9, and per-probe
    orthogonal tr(D^-1) terms within 1e-8 of |a| + |b|."""
    import paper_2509_11424_amd as m
    from oracle.dirac import WilsonClover
    from oracle.multigrid import Hierarchy
    from oracle.solve import level_solver
    from oracle import estimators as E
    ctx = m.Context(0)
    U = gauge_field((4, 4, 4, 4), 0.5, 12)
    op = m.Operator(ctx, U, 0.05, 1.0)
    h = m.Hierarchy(op, [(2, 2, 2, 2)], [64], seed=104, max_nrhs=16, restart=20, mixed=2)
    st = h.refine(max_iters=3, eig_tol=0.0, power_tol=1e-12, batch=16, solve=m.solve_desc(tol=1e-12))
    assert st["steps"] == 3 and st["converged"]
    D = WilsonClover(U, 0.05, 1.0)
    Dinv = np.linalg.inv(D.dense())
    oh = Hierarchy(D, [(2, 2, 2, 2)], [64], seed=104, refine=(lambda b: Dinv @ b, 3, 0.0))
    np.testing.assert_allclose(st["rho"], oh.refine_rho, rtol=1e-8)
    assert rel(h.export(0, "P"), oh.transfers[0].P) < 1e-9
    assert rel(h.export(0, "coarse"), oh.ops[1].blocks) < 1e-9
    solvers = [level_solver(o) for o in oh.ops]
    res = h.estimate("trace", "orthogonal", [3, 3], seed=31, batch=3, solve=m.solve_desc(tol=1e-12))
    want = [E.O_samples(oh, solvers, 0, 31, 3), E.F_samples(oh, solvers, 0, 31, 3),
            E.coarsest_samples(oh, solvers, 31, 3)]
    sc = np.abs(E.plain_samples(oh, solvers, 31, 1)[0])
    for q in range(3):
        got = res["samples"][q][:, 0, 0]
        assert np.all(np.abs(got - want[q]) <= 1e-8 * (np.abs(want[q]) + sc)), q


@pytest.fixture(scope="module")
def widest():
    """128 test vectors on 4 x 4 x 4 x 8 with aggregates of 2 x 2 x 2 x 4 sites
    (192 rows per block): a 16-site coarse level of 256 dof (sixteen MFMA row
    tiles), restrictions in rhs tiles of 32, FP64 prolongations in tiles of 16,
    Galerkin products in sixteen column chunks."""
    return _Pair((4, 4, 4, 8), 0.5, 68, 0.1, [(2, 2, 2, 4)], [128], 69, max_nrhs=40)


def test_128_vectors_P_coarse_and_transfers(widest):
    import torch
    from oracle.multigrid import Transfer
    p = widest
    assert p.h.level_info(1)[1] == 256
    assert np.array_equal(p.h.export(0, "agg_map"), p.oh.transfers[0].agg.block_index())
    assert rel(p.h.export(0, "P"), p.oh.transfers[0].P) < 1e-10
    assert rel(p.h.export(0, "coarse"), p.oh.ops[1].blocks) < 1e-10
    tr = p.oh.transfers[0]
    s, d, _ = p.h.level_info(0)
    cs, cd, _ = p.h.level_info(1)
    for nrhs in (1, 37):
        x = _rand(s, d, nrhs, 800 + nrhs)
        xc = _rand(cs, cd, nrhs, 900 + nrhs)
        xf, xcf = x.reshape(nrhs, -1), xc.reshape(nrhs, -1)
        assert rel(from_gpu(p.h.restrict(0, to_gpu(x))).reshape(nrhs, -1), tr.restrict(xf)) < 1e-10, nrhs
        assert rel(from_gpu(p.h.prolong(0, to_gpu(xc))).reshape(nrhs, -1), tr.prolong(xcf)) < 1e-10, nrhs
        assert rel(from_gpu(p.h.project_out(0, to_gpu(x))).reshape(nrhs, -1), tr.project_out(xf)) < 1e-10, nrhs
        re = tr.P.real.astype(np.float32).astype(np.float16).astype(np.float64)
        im = tr.P.imag.astype(np.float32).astype(np.float16).astype(np.float64)
        t16 = Transfer(tr.agg, re + 1j * im)
        x32, xc32 = x.astype(np.complex64), xc.astype(np.complex64)
        yc = p.h.restrict(0, to_gpu(x32).to(torch.complex64), prec="f32")
        y = p.h.prolong(0, to_gpu(xc32).to(torch.complex64), prec="f32")
        assert rel(from_gpu(yc).reshape(nrhs, -1), t16.restrict(x32.astype(np.complex128).reshape(nrhs, -1))) < 1e-5
        assert rel(from_gpu(y).reshape(nrhs, -1), t16.prolong(xc32.astype(np.complex128).reshape(nrhs, -1))) < 1e-5


def test_128_vectors_coarse_stencil(widest):
    """256-dof blocks: FP64 within 1e-10 of the oracle stencil, FP32 within
    2e-6, BF16 within 5e-5 of the BF16-rounded stencil, at 21 and 37 rhs."""
    import torch
    p = widest
    op = p.oh.ops[1]
    B, nbr = op.stencil()
    d, V = op.d, op.V
    g = np.where(np.arange(d) < d // 2, 1.0, -1.0)
    Bf = _bf16(B[:, :5].real) + 1j * _bf16(B[:, :5].imag)
    blocks = np.concatenate([Bf] + [
        (g[None, :, None] * np.conj(np.transpose(Bf[nbr[5 + mu], 1 + mu], (0, 2, 1))) * g[None, None, :])[:, None]
        for mu in range(4)], axis=1)
    for nrhs in (21, 37):
        x = _rand(V, d, nrhs, 700 + nrhs)
        got = p.h.apply_prec(1, to_gpu(x), "f64")
        assert rel(from_gpu(got).reshape(nrhs, -1), op.matvec(x.reshape(nrhs, -1))) < 1e-10
        x32 = x.astype(np.complex64)
        got = p.h.apply_prec(1, to_gpu(x32), "f32")
        want = op.matvec(x32.astype(np.complex128).reshape(nrhs, -1))
        assert rel(from_gpu(got).astype(np.complex128).reshape(nrhs, -1), want) < 2e-6
        xr = _bf16(x32.real) + 1j * _bf16(x32.imag)
        want = np.zeros((nrhs, V, d), dtype=np.complex128)
        for k in range(9):
            want += np.einsum("sij,nsj->nsi", blocks[:, k], xr[:, nbr[k], :])
        got = p.h.apply_prec(1, to_gpu(x32), "bf16")
        assert got.dtype == torch.complex64
        assert rel(from_gpu(got).astype(np.complex128).reshape(nrhs, -1), want.reshape(nrhs, -1)) < 5e-5


def test_128_vectors_solves_and_trace(widest):
    import torch
    import paper_2509_11424_amd as m
    from oracle import estimators as E
    p = widest
    for l in range(2):
        s, d, _ = p.h.level_info(l)
        b = _rand(s, d, 3, 90 + l)
        torch.cuda.synchronize()
        x, st = p.h.solve(l, to_gpu(b), m.solve_desc(tol=1e-12, kind="mg_mixed", maxiter=4000))
        torch.cuda.synchronize()
        assert st["max_rel_residual"] <= 1e-12, l
        want = np.stack([p.solvers[l](bb) for bb in b.reshape(3, -1)])
        assert rel(from_gpu(x).reshape(3, -1), want) < 1e-9, l
    seed, N = 77, 2
    res = p.h.estimate("trace", "orthogonal", [N, N], seed=seed, batch=2, solve=m.solve_desc(tol=1e-12))
    want = [E.O_samples(p.oh, p.solvers, 0, seed, N), E.F_samples(p.oh, p.solvers, 0, seed, N),
            E.coarsest_samples(p.oh, p.solvers, seed, N)]
    sc = np.abs(E.plain_samples(p.oh, p.solvers, seed, 1)[0])
    for q, w in enumerate(want):
        got = res["samples"][q][:, 0, 0]
        assert np.all(np.abs(got - w) <= 1e-8 * (np.abs(w) + sc)), (q, got, w)


@pytest.mark.parametrize("prec", ["bf16", "f32", "f64"])
def test_128_vectors_every_coarse_launch_shape(widest, prec):
    """Every launch shape the autotuner may pick for the 256-dof stencil at
    100 rhs (seven 16-rhs tiles): one, two or four waves per workgroup, one
    tile per wave (the wider shapes stop at eight row tiles)."""
    import torch
    p = widest
    op = p.oh.ops[1]
    B, nbr = op.stencil()
    d, V, nrhs = op.d, op.V, 100
    x = _rand(V, d, nrhs, 950)
    if prec != "f64":
        x = x.astype(np.complex64)
    if prec == "bf16":
        g = np.where(np.arange(d) < d // 2, 1.0, -1.0)
        Bf = _bf16(B[:, :5].real) + 1j * _bf16(B[:, :5].imag)
        blocks = np.concatenate([Bf] + [
            (g[None, :, None] * np.conj(np.transpose(Bf[nbr[5 + mu], 1 + mu], (0, 2, 1))) * g[None, None, :])[:, None]
            for mu in range(4)], axis=1)
        xr = _bf16(x.real) + 1j * _bf16(x.imag)
        want = np.zeros((nrhs, V, d), dtype=np.complex128)
        for k in range(9):
            want += np.einsum("sij,nsj->nsi", blocks[:, k], xr[:, nbr[k], :])
        want = want.reshape(nrhs, -1)
    else:
        want = op.matvec(x.astype(np.complex128).reshape(nrhs, -1))
    bar = {"bf16": 5e-5, "f32": 2e-6, "f64": 1e-10}[prec]
    tag = {"bf16": "coarsebf16", "f32": "coarse32", "f64": "coarse64"}[prec]
    key = "%s/%d/%d/%d" % (tag, V, d, nrhs)
    xg = to_gpu(x)
    p.ctx.autotune(True)
    try:
        p.h.apply_prec(1, xg, prec)
    finally:
        p.ctx.autotune(False)
    torch.cuda.synchronize()
    rep = p.ctx.tune_report()
    assert key in rep, (key, list(rep))
    nvar = len(rep[key][1])
    assert nvar == 3, (key, nvar)
    for v in range(nvar):
        p.ctx.tune_set(key, v)
        got = p.h.apply_prec(1, xg, prec)
        torch.cuda.synchronize()
        assert rel(from_gpu(got).astype(np.complex128).reshape(nrhs, -1), want) < bar, (key, v)
    p.ctx.tune_set(key, 0)
