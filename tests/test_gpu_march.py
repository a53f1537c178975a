"""Plane-marching fine dslash: a block keeps a tile of x-rows of one time
slice in LDS and registers while it marches along z.  Every launch shape that
applies to a lattice (tile rows, z-run, rhs group) is pinned in turn with
mgm_context_tune_set and checked

* against the site-parallel kernel (variant 0): the same per-hop arithmetic
  summed in another order, so FP32 agrees to a few units of FP32 rounding and
  FP16 (rounded once on store) to one FP16 ulp per element;
* against the oracle's operator within the storage precision's bound (the
  bounds of the site-parallel kernel's own parity tests);
* for the reducing variant, y^H x and |y|^2 against numpy's sums of the
  stored y (the kernel sums each site's twelve products in FP32, the sites in
  FP64: 1e-6 of ||y|| ||x||).

Lattices: 8x16x8x4 (one z-run covering the whole z extent, so the first plane's
backward neighbour wraps), 16x4x16x6 (two z-runs, T not a multiple of four)
and 8x8x32x4 (the 32-plane runs, one per time slice and tile).  The last
tests run the bench's launch configuration, 32^3 x 64: the reducing dslash at
eight FP16 right-hand sides against the FP64 dslash, and every launch variant
of the fused smoother step at 16, 8 and 4 right-hand sides against its
definition and the oracle's stencil at sampled sites.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from gpu_common import LocalStencil, to_gpu, from_gpu, rel  # noqa: E402
from lattice_inputs import gauge_field, random_spinor  # noqa: E402

BOUND = {"f32": 2e-6, "f16": 4e-3}


@pytest.fixture(scope="module")
def ctx():
    import paper_2509_11424_amd as m
    return m.Context(0)  # own context: pinned shapes must not leak into other tests


class Lat:
    def __init__(self, ctx, dims, seed):
        import paper_2509_11424_amd as m
        from oracle.dirac import WilsonClover
        self.dims = dims
        self.U = gauge_field(dims, 0.6, seed)
        self.op = m.Operator(ctx, self.U, 0.03, 1.0)
        self.D = WilsonClover(self.U, 0.03, 1.0)
        self.V = self.op.V


@pytest.fixture(scope="module")
def lats(ctx):
    return {"8x16x8x4": Lat(ctx, (8, 16, 8, 4), 41), "16x4x16x6": Lat(ctx, (16, 4, 16, 6), 42),
            "8x8x32x4": Lat(ctx, (8, 8, 32, 4), 44)}


def _inputs(lat, prec, nrhs, seed):
    import torch
    xs = random_spinor(lat.dims, seed, batch=nrhs)
    xg = to_gpu(xs.reshape(nrhs, -1, 12))
    if prec == "f32":
        return xs, xg.to(torch.complex64)
    return xs, torch.view_as_real(xg).to(torch.float16).contiguous()


def _c128(t, prec):
    import torch
    if prec == "f16":
        t = torch.view_as_complex(t.float().contiguous())
    return t.to(torch.complex128)


def _variants(ctx, key, run):
    """Tunes `key` once (listing its variants), returns the variant count."""
    ctx.autotune(True)
    try:
        run()
    finally:
        ctx.autotune(False)
    import torch
    torch.cuda.synchronize()
    rep = ctx.tune_report()
    assert key in rep, (key, list(rep))
    return len(rep[key][1])


def _close_to_site_parallel(y, y0, prec):
    a, b = y.cpu().numpy(), y0.cpu().numpy()
    if prec == "f32":
        assert rel(a, b) < 1e-6
        assert np.all(np.abs(a - b) <= 1e-5 * np.abs(b) + 1e-6 * np.abs(b).max())
    else:
        # one FP16 ulp (2^-10 relative) per element, plus the subnormal floor
        assert np.all(np.abs(a - b) <= 2.0 ** -10 * np.abs(b) + 2.0 ** -24 + 1e-7 * np.abs(b).max())


@pytest.mark.parametrize("lname", ["8x16x8x4", "16x4x16x6", "8x8x32x4"])
@pytest.mark.parametrize("prec", ["f32", "f16"])
@pytest.mark.parametrize("nrhs", [1, 4, 8])
def test_march_shapes_apply(ctx, lats, lname, prec, nrhs):
    import torch
    import paper_2509_11424_amd as m
    lat = lats[lname]
    xs, x = _inputs(lat, prec, nrhs, 50 + nrhs)
    key = "dslash/%d/%d/%d" % (m.api.PREC[prec], lat.V, nrhs)
    y = torch.empty_like(x)
    nvar = _variants(ctx, key, lambda: lat.op.apply(x, y, prec))
    ctx.tune_set(key, 0)
    y0 = lat.op.apply(x, prec=prec)
    torch.cuda.synchronize()
    want = lat.D.apply(xs).reshape(nrhs, -1, 12)
    n_march = 0
    for v in range(1, nvar):
        ctx.tune_set(key, v)
        yv = lat.op.apply(x, prec=prec)
        torch.cuda.synchronize()
        _close_to_site_parallel(yv, y0, prec)
        assert rel(from_gpu(_c128(yv, prec)), want) < BOUND[prec], v
        n_march += 1
    ctx.tune_set(key, 0)
    assert n_march >= 1  # every case here has at least one plane-marching shape


@pytest.mark.parametrize("lname", ["8x16x8x4", "16x4x16x6", "8x8x32x4"])
@pytest.mark.parametrize("prec,nrhs", [("f16", 8), ("f16", 4), ("f32", 4), ("f16", 1)])
def test_march_shapes_fused_reductions(ctx, lats, lname, prec, nrhs):
    import torch
    import paper_2509_11424_amd as m
    lat = lats[lname]
    xs, x = _inputs(lat, prec, nrhs, 70 + nrhs)
    key = "dslash_dot/%d/%d/%d" % (m.api.PREC[prec], lat.V, nrhs)
    nvar = _variants(ctx, key, lambda: lat.op.apply_dot(x, prec=prec))
    ctx.tune_set(key, 0)
    y0, _, _ = lat.op.apply_dot(x, prec=prec)
    torch.cuda.synchronize()
    want = lat.D.apply(xs).reshape(nrhs, -1, 12)
    xn = _c128(x, prec).cpu().numpy()
    assert nvar >= 3  # two site-parallel orders, then the plane-marching shapes
    for v in range(nvar):
        ctx.tune_set(key, v)
        y, yx, yy = lat.op.apply_dot(x, prec=prec)
        torch.cuda.synchronize()
        _close_to_site_parallel(y, y0, prec)
        yn = _c128(y, prec).cpu().numpy()
        assert rel(from_gpu(torch.from_numpy(yn)), want) < BOUND[prec], v
        for r in range(nrhs):
            a = np.vdot(yn[:, :, r].ravel(), xn[:, :, r].ravel())
            b = np.vdot(yn[:, :, r].ravel(), yn[:, :, r].ravel()).real
            nx = np.linalg.norm(xn[:, :, r])
            assert abs(yx[r].item() - a) <= 1e-6 * np.sqrt(b) * nx, (v, r)
            assert abs(yy[r].item() - b) <= 1e-6 * b, (v, r)
    ctx.tune_set(key, 0)


@pytest.fixture(scope="module")
def full(ctx):
    """The bench's fine lattice, 32^3 x 64 (roughness 0.6, m0 0.02, c_sw 1)."""
    import paper_2509_11424_amd as m
    U = gauge_field((32, 32, 32, 64), 0.6, 14)
    return U, m.Operator(ctx, U, 0.02, 1.0)


def test_march_full_size_f16_eight_rhs(ctx, full):
    """32^3 x 64 at eight FP16 right-hand sides: every shape of the reducing
    dslash against the FP64 dslash of the same rounded input and against
    variant 0, and its dots against torch's sums."""
    import torch
    import paper_2509_11424_amd as m
    U, op = full
    V, nrhs = op.V, 8
    g = torch.Generator(device="cuda:0").manual_seed(3)
    x = torch.randn((12, V, nrhs, 2), generator=g, device="cuda:0").to(torch.float16)
    xc = torch.view_as_complex(x.float().contiguous()).to(torch.complex128)
    ref = op.apply(xc, prec="f64")
    key = "dslash_dot/%d/%d/%d" % (m.api.PREC["f16"], V, nrhs)
    nvar = _variants(ctx, key, lambda: op.apply_dot(x, prec="f16"))
    assert nvar >= 3
    ctx.tune_set(key, 0)
    y0, _, _ = op.apply_dot(x, prec="f16")
    y0c = torch.view_as_complex(y0.float().contiguous()).to(torch.complex128)
    for v in range(nvar):
        ctx.tune_set(key, v)
        y, yx, yy = op.apply_dot(x, prec="f16")
        yc = torch.view_as_complex(y.float().contiguous()).to(torch.complex128)
        d = (yc - ref).norm() / ref.norm()
        assert d.item() < BOUND["f16"], v
        # per element within one FP16 ulp of variant 0
        bad = ((yc - y0c).abs() > 2.0 ** -9 * y0c.abs() + 1e-6).sum().item()
        assert bad == 0, (v, bad)
        a = (yc.conj() * xc).sum(dim=(0, 1))
        b = (yc.abs() ** 2).sum(dim=(0, 1))
        nx = (xc.abs() ** 2).sum(dim=(0, 1)).sqrt()
        assert torch.all((yx - a).abs() <= 1e-6 * b.sqrt() * nx), v
        assert torch.all((yy - b).abs() <= 1e-6 * b), v
    ctx.tune_set(key, 0)
    # variant 0 against the oracle's stencil at sampled sites (FP64, from the
    # definition, on the stored FP16 input): FP16 links, clover and output
    # give at most 4e-3 of the site's norm
    xs_np = xc[:, :, :2].cpu().numpy()  # (12, V, 2)
    y0_np = y0c[:, :, :2].cpu().numpy()
    st = LocalStencil(U, 0.02, 1.0)
    rng = np.random.default_rng(7)
    for s_ in rng.integers(0, V, 12):
        for r in range(2):
            want = st.at(s_, xs_np[:, :, r].T)
            assert np.linalg.norm(y0_np[:, s_, r] - want) <= 4e-3 * np.linalg.norm(want), (s_, r)
    del x, xc, ref, y0, y0c
    torch.cuda.empty_cache()


@pytest.mark.parametrize("lname", ["8x16x8x4", "16x4x16x6", "8x8x32x4"])
@pytest.mark.parametrize("nrhs", [16, 4, 6, 1])
def test_fused_smoother_step(ctx, lats, lname, nrhs):
    """mgm_operator_smoother_step in every launch variant: the marching
    shapes with FP32 arithmetic on converted values, then the same shapes
    with packed FP16 arithmetic.

    FP32 form against its definition built from the reducing dslash: q = D r,
    r' = r - omega q, x' = x + omega r with omega = qr / qq of the previous
    step (0 where qq = 0), and the dots of (q, r); r' and x' within one FP16
    ulp plus omega times the FP16 rounding of q (the kernel uses q before
    rounding); dots within 1e-4 of those of the rounded q.

    Packed form: x' as above (the same FP32 update); q differs from the FP32
    form's by the FP16 rounding of the half spinors (2^-11 of each hop), so r'
    is checked norm-wise, within 2^-10 |r'| + 2e-3 |omega| |q| of the FP32
    form's, and the dots within 2e-3.

    Both against the oracle: q = D r from the FP64 operator on the stored FP16
    r, r' and the dots within the FP16 operator's bound (4e-3 of |q|)."""
    import torch
    import paper_2509_11424_amd as m
    lat = lats[lname]
    op = lat.op
    assert op.step_fusable(nrhs)
    g = torch.Generator(device="cuda:0").manual_seed(90 + nrhs)
    shape = (12, lat.V, nrhs, 2)
    r, x0 = (torch.randn(shape, generator=g, device="cuda:0").to(torch.float16) for _ in range(2))
    qr = torch.complex(torch.randn(nrhs, generator=g, device="cuda:0", dtype=torch.float64),
                       torch.randn(nrhs, generator=g, device="cuda:0", dtype=torch.float64)) * 0.05
    qq = torch.rand(nrhs, generator=g, device="cuda:0", dtype=torch.float64) + 0.5
    if nrhs > 1:
        qq[0] = 0.0  # omega = 0 for the first rhs
    key = "dslash_step/%d/%d/%d" % (m.api.PREC["f16"], lat.V, nrhs)
    nvar = _variants(ctx, key, lambda: op.smoother_step(r, x0.clone(), qr, qq))
    assert nvar % 2 == 0 and nvar >= 2
    ns = nvar // 2
    q, yx_ref, yy_ref = op.apply_dot(r, prec="f16")
    torch.cuda.synchronize()

    def c(t):
        return torch.view_as_complex(t.float().contiguous()).to(torch.complex128)

    om = torch.where(qq > 0, qr / qq.clamp_min(1e-300), torch.zeros_like(qr))
    want_x = c(x0) + om * c(r)
    nr = c(r).abs().pow(2).sum(dim=(0, 1)).sqrt()
    rr = from_gpu(c(r)).reshape(nrhs, -1)
    qo = lat.D.matvec(rr)
    omn = om.cpu().numpy()
    out = {}
    for v in range(nvar):
        packed = v >= ns
        ctx.tune_set(key, v)
        x = x0.clone()
        rn, yx, yy = op.smoother_step(r, x, qr, qq)
        torch.cuda.synchronize()
        out[v] = (rn, yx, yy)
        assert torch.all((c(x) - want_x).abs() <= 2.0 ** -10 * want_x.abs() + 2.0 ** -14 + 1e-6), v
        if nrhs > 1:
            assert torch.equal(rn[:, :, 0], r[:, :, 0]) and torch.equal(x[:, :, 0], x0[:, :, 0]), v
        if not packed:
            want_r = c(r) - om * c(q)
            slack = om.abs() * c(q).abs() * 2.0 ** -10
            assert torch.all((c(rn) - want_r).abs() <= 2.0 ** -10 * want_r.abs() + slack + 2.0 ** -14 + 1e-6), v
            assert torch.all((yx - yx_ref).abs() <= 1e-4 * yy_ref.sqrt() * nr), v
            assert torch.all((yy - yy_ref).abs() <= 1e-4 * yy_ref), v
        else:
            rn32, yx32, yy32 = out[v - ns]
            d = (c(rn) - c(rn32)).abs().pow(2).sum(dim=(0, 1)).sqrt()
            nq = c(q).abs().pow(2).sum(dim=(0, 1)).sqrt()
            nrn = c(rn32).abs().pow(2).sum(dim=(0, 1)).sqrt()
            assert torch.all(d <= 2.0 ** -10 * nrn + 2e-3 * om.abs() * nq + 1e-6), v
            assert torch.all((yx - yx32).abs() <= 2e-3 * yy32.sqrt() * nr), v
            assert torch.all((yy - yy32).abs() <= 4e-3 * yy32), v
        rn_np = from_gpu(c(rn)).reshape(nrhs, -1)
        yxn, yyn = yx.cpu().numpy(), yy.cpu().numpy()
        for j in range(nrhs):
            want_rj = rr[j] - omn[j] * qo[j]
            nqj = np.linalg.norm(qo[j])
            assert np.linalg.norm(rn_np[j] - want_rj) <= 2.0 ** -10 * np.linalg.norm(want_rj) + \
                abs(omn[j]) * 4e-3 * nqj, (v, j)
            assert abs(yxn[j] - np.vdot(qo[j], rr[j])) <= 4e-3 * nqj * np.linalg.norm(rr[j]), (v, j)
            assert abs(yyn[j] - nqj ** 2) <= 8e-3 * nqj ** 2, (v, j)
    del out
    ctx.tune_set(key, 0)


def test_fused_smoother_step_refuses_lattice_without_tile(ctx):
    import torch
    import paper_2509_11424_amd as m
    U = gauge_field((4, 4, 4, 8), 0.6, 43)
    op = m.Operator(ctx, U, 0.03, 1.0)
    assert not op.step_fusable(4)
    t = torch.zeros((12, op.V, 4, 2), dtype=torch.float16, device="cuda:0")
    z = torch.zeros(4, dtype=torch.complex128, device="cuda:0")
    with pytest.raises(RuntimeError, match="SHAPE"):
        op.smoother_step(t, t.clone(), z, torch.ones(4, dtype=torch.float64, device="cuda:0"))


@pytest.mark.parametrize("nrhs", [16, 8, 4])
def test_fused_smoother_step_full_size(ctx, full, nrhs):
    """32^3 x 64 at the rhs counts of the bench's fine level (a batch of 16,
    smoothed in column groups of 8, and 4 for the rest of 20 probes): every
    launch variant of the fused smoother step, among them the 32-plane
    shapes the bench runs.

    x' = x + omega r within one FP16 ulp of the update; FP32 forms: r' = r -
    omega q per element against q from the reducing FP16 dslash (slack for
    its rounding, as on the small lattices) and the dots within 1e-4; packed
    forms: r' norm-wise and the dots within 2e-3 of the FP32 form of the same
    shape; every variant: r' at 12 sampled sites and two rhs against r - omega
    q with q from the oracle's stencil on the stored FP16 r (FP64), within the
    FP16 operator's bound (4e-3 of |q|) plus one FP16 ulp of r'."""
    import torch
    import paper_2509_11424_amd as m
    U, op = full
    V = op.V
    g = torch.Generator(device="cuda:0").manual_seed(190 + nrhs)
    shape = (12, V, nrhs, 2)
    r, x0 = (torch.randn(shape, generator=g, device="cuda:0").to(torch.float16) for _ in range(2))
    qr = torch.complex(torch.randn(nrhs, generator=g, device="cuda:0", dtype=torch.float64),
                       torch.randn(nrhs, generator=g, device="cuda:0", dtype=torch.float64)) * 0.05
    qq = torch.rand(nrhs, generator=g, device="cuda:0", dtype=torch.float64) + 0.5
    key = "dslash_step/%d/%d/%d" % (m.api.PREC["f16"], V, nrhs)
    nvar = _variants(ctx, key, lambda: op.smoother_step(r, x0.clone(), qr, qq))
    assert nvar % 2 == 0 and nvar >= 2
    ns = nvar // 2
    q, yx_ref, yy_ref = op.apply_dot(r, prec="f16")
    torch.cuda.synchronize()

    def c(t):
        return torch.view_as_complex(t.float().contiguous())

    def n2(t):  # per-rhs squared norms, summed in FP64
        return t.abs().double().pow(2).sum(dim=(0, 1))

    om = torch.where(qq > 0, qr / qq, torch.zeros_like(qr))
    om32 = om.to(torch.complex64)
    want_x = c(x0) + om32 * c(r)
    nr, nq = n2(c(r)).sqrt(), n2(c(q)).sqrt()
    # oracle q at sampled sites for the first two rhs
    st = LocalStencil(U, 0.02, 1.0)
    sites = np.random.default_rng(11).integers(0, V, 12)
    rs = [c(r)[:, :, j].to(torch.complex128).cpu().numpy().T for j in range(2)]  # (V, 12)
    qs = [[st.at(s_, rs[j]) for s_ in sites] for j in range(2)]
    omn = om.cpu().numpy()
    out = {}
    for v in range(nvar):
        packed = v >= ns
        ctx.tune_set(key, v)
        x = x0.clone()
        rn, yx, yy = op.smoother_step(r, x, qr, qq)
        torch.cuda.synchronize()
        assert torch.all((c(x) - want_x).abs() <= 2.0 ** -10 * want_x.abs() + 2.0 ** -14 + 1e-6), v
        del x
        if not packed:
            want_r = c(r) - om32 * c(q)
            slack = om32.abs() * c(q).abs() * 2.0 ** -10
            assert torch.all((c(rn) - want_r).abs() <= 2.0 ** -10 * want_r.abs() + slack + 2.0 ** -14 + 1e-6), v
            del want_r, slack
            assert torch.all((yx - yx_ref).abs() <= 1e-4 * yy_ref.sqrt() * nr), v
            assert torch.all((yy - yy_ref).abs() <= 1e-4 * yy_ref), v
            out[v] = (rn, yx, yy)
        else:
            rn32, yx32, yy32 = out.pop(v - ns)
            d = n2(c(rn) - c(rn32)).sqrt()
            assert torch.all(d <= 2.0 ** -10 * n2(c(rn32)).sqrt() + 2e-3 * om.abs() * nq + 1e-6), v
            assert torch.all((yx - yx32).abs() <= 2e-3 * yy32.sqrt() * nr), v
            assert torch.all((yy - yy32).abs() <= 4e-3 * yy32), v
        for j in range(2):
            rnj = c(rn)[:, :, j].to(torch.complex128).cpu().numpy().T
            for k, s_ in enumerate(sites):
                want = rs[j][s_] - omn[j] * qs[j][k]
                assert np.linalg.norm(rnj[s_] - want) <= 2.0 ** -10 * np.linalg.norm(want) + \
                    abs(omn[j]) * 4e-3 * np.linalg.norm(qs[j][k]) + 1e-6, (v, j, s_)
    out.clear()
    ctx.tune_set(key, 0)
    del r, x0, q, want_x
    torch.cuda.empty_cache()
