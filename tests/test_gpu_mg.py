"""GPU parity of the multigrid hierarchy, solves and estimators against the
FP64 oracle.

Bars: aggregation maps bit-exact; P, D_c and test vectors within 1e-10
relative (20 x 4 minimal-residual rounds amplify rounding-order differences
by at most a few hundred ulps); solutions within 1e-9 of a dense solve at
tol 1e-12; per-probe quadratic forms within 1e-8 relative, with differences
X = a - b measured against |a| + |b|.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from gpu_common import to_gpu, from_gpu, rel  # noqa: E402
from lattice_inputs import gauge_field, random_spinor  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    import paper_2509_11424_amd as m
    return m.Context(0)


class Pair:
    """GPU hierarchy and oracle hierarchy on the same inputs."""

    def __init__(self, ctx, dims, eps, gseed, m0, csw, blocks, ntv, seed, max_nrhs=8, with_corr=False,
                 mixed=0):
        import paper_2509_11424_amd as m
        from oracle.dirac import WilsonClover
        from oracle.multigrid import Hierarchy
        from oracle.solve import level_solver
        self.U = gauge_field(dims, eps, gseed)
        self.op = m.Operator(ctx, self.U, m0, csw)
        self.h = m.Hierarchy(self.op, blocks, ntv, seed=seed, max_nrhs=max_nrhs, restart=20,
                             with_corr=with_corr, mixed=mixed)
        self.D = WilsonClover(self.U, m0, csw)
        self.oh = Hierarchy(self.D, blocks, ntv, seed=seed)
        self.solvers = [level_solver(o) for o in self.oh.ops]


@pytest.fixture(scope="module")
def two(ctx):
    return Pair(ctx, (4, 4, 4, 4), 0.5, 12, 0.05, 1.0, [(2, 2, 2, 2)], [8], 102, with_corr=True)


@pytest.fixture(scope="module")
def three(ctx):
    return Pair(ctx, (4, 4, 4, 8), 0.5, 21, 0.1, 1.0, [(2, 2, 2, 2), (1, 1, 1, 2)], [6, 4], 7,
                with_corr=True)


def test_test_vectors_match(two):
    tv = two.h.export(0, "tv")
    assert rel(tv, two.oh.tvs[0]) < 1e-10


def test_aggregation_map_bit_exact(two, three):
    for p in (two, three):
        for l in range(p.oh.L - 1):
            assert np.array_equal(p.h.export(l, "agg_map"), p.oh.transfers[l].agg.block_index())


def test_P_and_coarse_operator(two, three):
    for p in (two, three):
        for l in range(p.oh.L - 1):
            assert rel(p.h.export(l, "P"), p.oh.transfers[l].P) < 1e-10
            assert rel(p.h.export(l, "coarse"), p.oh.ops[l + 1].blocks) < 1e-10


def _rand(n_site, dof, nrhs, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((nrhs, n_site, dof)) + 1j * rng.standard_normal((nrhs, n_site, dof))


def test_transfers_and_level_apply(three):
    p = three
    for l in range(p.oh.L - 1):
        s, d, n = p.h.level_info(l)
        cs, cd, cn = p.h.level_info(l + 1)
        x = _rand(s, d, 3, l)
        xc = _rand(cs, cd, 3, 10 + l)
        tr = p.oh.transfers[l]
        xf, xcf = x.reshape(3, -1), xc.reshape(3, -1)
        assert rel(from_gpu(p.h.restrict(l, to_gpu(x))).reshape(3, -1), tr.restrict(xf)) < 1e-10
        assert rel(from_gpu(p.h.prolong(l, to_gpu(xc))).reshape(3, -1), tr.prolong(xcf)) < 1e-10
        assert rel(from_gpu(p.h.project_out(l, to_gpu(x))).reshape(3, -1), tr.project_out(xf)) < 1e-10
    for l in range(p.oh.L):
        s, d, n = p.h.level_info(l)
        x = _rand(s, d, 2, 20 + l)
        y = from_gpu(p.h.apply(l, to_gpu(x))).reshape(2, -1)
        assert rel(y, p.oh.ops[l].matvec(x.reshape(2, -1))) < 1e-10


@pytest.fixture(scope="module")
def wide(ctx):
    """24 and 32 test vectors, aggregates of 32 and 2 sites: transfer blocks of
    192 and 48 rows that span several LDS chunks, in a mixed hierarchy."""
    return Pair(ctx, (4, 4, 4, 16), 0.5, 33, 0.1, 1.0, [(2, 2, 2, 4), (1, 1, 1, 2)], [24, 32], 41,
                max_nrhs=72, mixed=1)


@pytest.mark.parametrize("nrhs", [1, 5, 70])
def test_transfers_many_vectors_f64(wide, nrhs):
    p = wide
    for l in range(p.oh.L - 1):
        s, d, n = p.h.level_info(l)
        cs, cd, cn = p.h.level_info(l + 1)
        x = _rand(s, d, nrhs, 100 + l)
        xc = _rand(cs, cd, nrhs, 200 + l)
        tr = p.oh.transfers[l]
        xf, xcf = x.reshape(nrhs, -1), xc.reshape(nrhs, -1)
        assert rel(from_gpu(p.h.restrict(l, to_gpu(x))).reshape(nrhs, -1), tr.restrict(xf)) < 1e-10
        assert rel(from_gpu(p.h.prolong(l, to_gpu(xc))).reshape(nrhs, -1), tr.prolong(xcf)) < 1e-10
        assert rel(from_gpu(p.h.project_out(l, to_gpu(x))).reshape(nrhs, -1), tr.project_out(xf)) < 1e-10


def _fp16_rounded(P):
    """P as the mixed transfers hold it: FP64 -> FP32 -> FP16, per component."""
    re = P.real.astype(np.float32).astype(np.float16).astype(np.float64)
    im = P.imag.astype(np.float32).astype(np.float16).astype(np.float64)
    return re + 1j * im


@pytest.mark.parametrize("nrhs", [3, 16, 70])
def test_transfers_f32_fp16_P(wide, nrhs):
    """FP32 transfers with FP16-stored P against the oracle's P rounded the
    same way, applied in FP64 to the same FP32 inputs: only FP32 accumulation
    (at most 192 terms) separates the two."""
    import torch
    from oracle.multigrid import Transfer
    p = wide
    for l in range(p.oh.L - 1):
        s, d, n = p.h.level_info(l)
        cs, cd, cn = p.h.level_info(l + 1)
        x = _rand(s, d, nrhs, 300 + l).astype(np.complex64)
        xc = _rand(cs, cd, nrhs, 400 + l).astype(np.complex64)
        tr = p.oh.transfers[l]
        t16 = Transfer(tr.agg, _fp16_rounded(tr.P))
        yc = p.h.restrict(l, to_gpu(x).to(torch.complex64), prec="f32")
        y = p.h.prolong(l, to_gpu(xc).to(torch.complex64), prec="f32")
        assert yc.dtype == torch.complex64 and y.dtype == torch.complex64
        want_c = t16.restrict(x.astype(np.complex128).reshape(nrhs, -1))
        want = t16.prolong(xc.astype(np.complex128).reshape(nrhs, -1))
        assert rel(from_gpu(yc).reshape(nrhs, -1), want_c) < 1e-5
        assert rel(from_gpu(y).reshape(nrhs, -1), want) < 1e-5


def _bf16(a):
    """round to nearest even BF16 after rounding to FP32 (as the device does)"""
    b = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def _bf16c(z):
    return _bf16(z.real) + 1j * _bf16(z.imag)


@pytest.mark.parametrize("nrhs", [4, 37])
def test_coarse_bf16_backward_blocks(wide, nrhs):
    """BF16 coarse stencil against an FP64 stencil built from the oracle's
    self and forward blocks rounded to BF16, with every backward block the
    chirality-signed conjugate transpose of the neighbour's rounded forward
    block (gamma5-hermiticity; round-to-nearest-even commutes with sign
    changes, so this equals the rounded backward block), on BF16-rounded
    inputs: only the FP32 accumulation separates the two.  d = 48 and 64
    (three and four 16-row tiles, chirality boundary inside and at the edge
    of a tile)."""
    import torch
    p = wide
    for l in (1, 2):
        op = p.oh.ops[l]
        B, nbr = op.stencil()
        d, V = op.d, op.V
        g = np.where(np.arange(d) < d // 2, 1.0, -1.0)
        Bf = _bf16c(B[:, :5])
        blocks = np.concatenate([Bf] + [
            (g[None, :, None] * np.conj(np.transpose(Bf[nbr[5 + mu], 1 + mu], (0, 2, 1))) * g[None, None, :])[:, None]
            for mu in range(4)], axis=1)
        x = _rand(V, d, nrhs, 500 + l).astype(np.complex64)
        xr = _bf16c(x.astype(np.complex128))
        want = np.zeros((nrhs, V, d), dtype=np.complex128)
        for k in range(9):
            want += np.einsum("sij,nsj->nsi", blocks[:, k], xr[:, nbr[k], :])
        got = p.h.apply_prec(l, to_gpu(x), "bf16")
        assert rel(from_gpu(got).astype(np.complex128).reshape(nrhs, -1), want.reshape(nrhs, -1)) < 5e-5


def _coarse_want(op, x, prec):
    """Reference of the level-l stencil in precision prec for input x."""
    if prec != "bf16":
        return op.matvec(x.astype(np.complex128).reshape(x.shape[0], -1))
    B, nbr = op.stencil()
    d = op.d
    g = np.where(np.arange(d) < d // 2, 1.0, -1.0)
    Bf = _bf16c(B[:, :5])
    blocks = np.concatenate([Bf] + [
        (g[None, :, None] * np.conj(np.transpose(Bf[nbr[5 + mu], 1 + mu], (0, 2, 1))) * g[None, None, :])[:, None]
        for mu in range(4)], axis=1)
    xr = _bf16c(x.astype(np.complex128))
    want = np.zeros(x.shape, dtype=np.complex128)
    for k in range(9):
        want += np.einsum("sij,nsj->nsi", blocks[:, k], xr[:, nbr[k], :])
    return want.reshape(x.shape[0], -1)


@pytest.mark.parametrize("prec", ["bf16", "f32", "f64"])
@pytest.mark.parametrize("nrhs", [37, 100])
def test_coarse_stencil_every_launch_shape(ctx, wide, prec, nrhs):
    """Every launch shape the autotuner may pick for the coarse stencils
    (waves per workgroup, tiles per wave, all of a site's tiles in one
    workgroup) against the oracle: f64 within 1e-10 (the bar of D_c), f32
    within 2e-6, bf16 within 5e-5 of the BF16-rounded stencil."""
    import torch
    p = wide
    tag = {"bf16": "coarsebf16", "f32": "coarse32", "f64": "coarse64"}[prec]
    bar = {"bf16": 5e-5, "f32": 2e-6, "f64": 1e-10}[prec]
    for l in (1, 2):
        op = p.oh.ops[l]
        x = _rand(op.V, op.d, nrhs, 600 + l)
        if prec != "f64":
            x = x.astype(np.complex64)
        xg = to_gpu(x)
        want = _coarse_want(op, x, prec)
        key = "%s/%d/%d/%d" % (tag, op.V, op.d, nrhs)
        ctx.autotune(True)
        try:
            p.h.apply_prec(l, xg, prec)
        finally:
            ctx.autotune(False)
        torch.cuda.synchronize()
        rep = ctx.tune_report()
        assert key in rep, (key, list(rep))
        nvar = len(rep[key][1])
        if nrhs == 100:  # seven tiles: the whole-site shapes are among the candidates
            assert nvar >= (4 if prec != "bf16" else 7), (key, nvar)
        for v in range(nvar):
            ctx.tune_set(key, v)
            got = p.h.apply_prec(l, xg, prec)
            torch.cuda.synchronize()
            assert rel(from_gpu(got).astype(np.complex128).reshape(nrhs, -1), want) < bar, (key, v)
        ctx.tune_set(key, 0)


def _f16_pairs(x):
    """numpy (nrhs, sites, dof) complex -> device float16 pairs (dof, sites, nrhs, 2)
    and the values they hold as complex128 (nrhs, sites, dof)"""
    import torch
    from paper_2509_11424_amd import to_dofmajor
    xd = to_dofmajor(x)
    pairs = np.stack([xd.real, xd.imag], axis=-1).astype(np.float16)
    held = pairs[..., 0].astype(np.float64) + 1j * pairs[..., 1].astype(np.float64)
    return torch.from_numpy(np.ascontiguousarray(pairs)).to("cuda:0"), np.transpose(held, (2, 1, 0))


@pytest.mark.parametrize("nrhs", [3, 16, 70])
def test_transfers_fp16_input(wide, nrhs):
    """Transfers of the mixed V-cycle that read the FP16 smoother vectors
    with per-rhs scales: y_c = P^H (s x16) and y = s x16 + P x_c, against the
    oracle's P rounded to FP16 applied in FP64 to the values the FP16 input
    holds (FP32 accumulation only)."""
    import torch
    from oracle.multigrid import Transfer
    p = wide
    rng = np.random.default_rng(900 + nrhs)
    scale = rng.uniform(0.1, 10.0, nrhs)
    sg = torch.from_numpy(scale).to("cuda:0")
    for l in range(p.oh.L - 1):
        s, d, n = p.h.level_info(l)
        cs, cd, cn = p.h.level_info(l + 1)
        x16, held = _f16_pairs(_rand(s, d, nrhs, 600 + l))
        xc = _rand(cs, cd, nrhs, 700 + l).astype(np.complex64)
        t16 = Transfer(p.oh.transfers[l].agg, _fp16_rounded(p.oh.transfers[l].P))
        xs = (scale[:, None, None] * held).reshape(nrhs, -1)
        yc = p.h.restrict_f16(l, x16, sg)
        assert rel(from_gpu(yc).reshape(nrhs, -1), t16.restrict(xs)) < 1e-5
        y = p.h.prolong_add_f16(l, to_gpu(xc), x16, sg)
        want = xs + t16.prolong(xc.astype(np.complex128).reshape(nrhs, -1))
        assert rel(from_gpu(y).reshape(nrhs, -1), want) < 1e-5


def test_transfer_prec_rejects_f16(wide):
    import torch
    import paper_2509_11424_amd as m
    s, d, n = wide.h.level_info(0)
    x = torch.zeros((d, s, 2), dtype=torch.complex64, device="cuda:0")
    with pytest.raises(m.MgmError):
        wide.h.restrict(0, x, prec="f16")


@pytest.mark.parametrize("kind", ["mg", "gmres"])
def test_solves_every_level(three, kind):
    import paper_2509_11424_amd as m
    p = three
    for l in range(p.oh.L):
        s, d, n = p.h.level_info(l)
        b = _rand(s, d, 3, 30 + l)
        x, st = p.h.solve(l, to_gpu(b), m.solve_desc(tol=1e-12, kind=kind, maxiter=3000))
        assert st["max_rel_residual"] <= 1e-12
        want = np.stack([p.solvers[l](bb) for bb in b.reshape(3, -1)])
        assert rel(from_gpu(x).reshape(3, -1), want) < 1e-9


def _close(got, want, scale, tol=1e-8):
    return np.all(np.abs(got - want) <= tol * scale)


@pytest.mark.parametrize("dec", ["plain", "oblique", "orthogonal"])
def test_trace_per_probe(two, three, dec):
    import paper_2509_11424_amd as m
    from oracle import estimators as E
    for p in (two, three):
        L = p.oh.L
        npr = [3] * L
        res = p.h.estimate("trace", dec, npr, seed=55, batch=2, solve=m.solve_desc(tol=1e-12))
        S = res["samples"]
        if dec == "plain":
            want = [E.plain_samples(p.oh, p.solvers, 55, 3)]
        elif dec == "oblique":
            want = [E.M_samples(p.oh, p.solvers, l, 55, 3) for l in range(L - 1)]
            want += [E.coarsest_samples(p.oh, p.solvers, 55, 3)]
        else:
            want = [E.O_samples(p.oh, p.solvers, l, 55, 3) for l in range(L - 1)]
            want += [E.F_samples(p.oh, p.solvers, l, 55, 3) for l in range(L - 1)]
            want += [E.coarsest_samples(p.oh, p.solvers, 55, 3)]
        assert len(S) == len(want)
        for q in range(len(want)):
            got = S[q][:, 0, 0]
            # difference terms: error relative to |a| + |b| (scale by the plain magnitude)
            scale = np.abs(want[q]) + np.abs(E.plain_samples(p.oh, p.solvers, 55, 1)[0])
            assert _close(got, want[q], scale), (dec, q, got, want[q])
        # means and variances from the returned samples
        for q in range(len(want)):
            mu, var = E.mean_var(S[q][:, 0, 0])
            assert abs(res["mean"][q, 0, 0] - mu) <= 1e-12 * abs(mu) + 1e-14
            assert abs(res["var"][q, 0, 0] - var) <= 1e-9 * var + 1e-14


@pytest.mark.parametrize("dec", ["plain", "oblique", "orthogonal"])
def test_correlator_per_probe(two, three, dec):
    import paper_2509_11424_amd as m
    from oracle import estimators as E
    for p in (two, three):
        L = p.oh.L
        R = len(E.term_levels(L, dec))
        res = p.h.estimate("corr", dec, [2] * L, seed=77, batch=2, solve=m.solve_desc(tol=1e-12))
        groups = [0] if dec == "plain" else range(L)
        for g in groups:
            pairs, X = E.correlator_samples(p.oh, p.solvers, dec, g, seed=77, nprobe=2)
            for ip, (r, s) in enumerate(pairs):
                got = res["samples"][r * R + s][:, 0, :]
                scale = np.abs(X[:, ip, :]).max() + 1e-300
                assert np.abs(got - X[:, ip, :]).max() <= 1e-8 * scale, (dec, g, r, s)


@pytest.mark.parametrize("dec", ["plain", "oblique", "orthogonal"])
def test_loops_per_probe(two, three, dec):
    """Loop slices tr(Gamma B(t,t)) per probe, term, Gamma and t (Sec. 4.3)
    on two- and three-level hierarchies against the oracle."""
    import paper_2509_11424_amd as m
    from oracle import estimators as E
    for p in (two, three):
        L = p.oh.L
        res = p.h.estimate("loops", dec, [3] * L, seed=5, batch=3, solve=m.solve_desc(tol=1e-12))
        groups = [0] if dec == "plain" else range(L)
        for g in groups:
            terms, X = E.loop_samples(p.oh, p.solvers, dec, g, seed=5, nprobe=3)
            for it, r in enumerate(terms):
                got = res["samples"][r]
                scale = np.abs(X[:, it]).max()
                assert np.abs(got - X[:, it]).max() <= 1e-8 * scale, (L, dec, g, r)


def test_estimate_first_probe_offset_reproduces(two):
    """Probe k of a run starting at first_probe = 2 equals probe 2 + k of a run from 0."""
    import paper_2509_11424_amd as m
    sd = m.solve_desc(tol=1e-12)
    a = two.h.estimate("trace", "orthogonal", [4, 4], seed=9, batch=4, solve=sd)
    b = two.h.estimate("trace", "orthogonal", [2, 2], seed=9, batch=2, first_probe=2, solve=sd)
    for q in range(3):
        np.testing.assert_allclose(b["samples"][q][:, 0, 0], a["samples"][q][2:, 0, 0], rtol=1e-9)


def test_not_converged_reports_status(two):
    import paper_2509_11424_amd as m
    s, d, n = two.h.level_info(0)
    b = _rand(s, d, 1, 3)
    x, st = two.h.solve(0, to_gpu(b), m.solve_desc(tol=1e-12, kind="gmres", maxiter=3), check=False)
    assert st["status"] == -4 and st["max_rel_residual"] > 1e-12


def test_nan_input_reports_numeric(two):
    import paper_2509_11424_amd as m
    s, d, n = two.h.level_info(0)
    b = _rand(s, d, 1, 3)
    b[0, 0, 0] = np.nan
    with pytest.raises(m.MgmError) as e:
        two.h.solve(0, to_gpu(b), m.solve_desc(tol=1e-12))
    assert e.value.status == -6
