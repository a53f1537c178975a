"""The allocation-free reducing dslash (mgm_operator_apply_dot_noalloc).

It runs the kernels of mgm_operator_apply_dot with the reduction partials in
the library's fixed device array instead of a caller workspace, so its
outputs must equal that entry point's bit for bit.  Two calls in a row, the
second with a smaller input, check that the shared array keeps no state that
matters between calls; the outputs are also checked against the oracle's
operator.  A shape whose partials exceed the array is refused before any
launch.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from gpu_common import to_gpu, from_gpu, rel  # noqa: E402
from lattice_inputs import gauge_field, random_spinor  # noqa: E402

BOUND = {"f64": 1e-13, "f32": 2e-6, "f16": 4e-3}


def _as_prec(xc, prec):
    import torch
    if prec == "f64":
        return xc
    if prec == "f32":
        return xc.to(torch.complex64)
    return torch.view_as_real(xc).to(torch.float16).contiguous()


def _c128(t, prec):
    import torch
    if prec == "f16":
        return torch.view_as_complex(t.float().contiguous()).to(torch.complex128)
    return t.to(torch.complex128)


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_noalloc_matches_workspace_entry_point(prec):
    import torch
    import paper_2509_11424_amd as m
    from oracle.dirac import WilsonClover
    ctx = m.Context(0)
    dims = (8, 16, 8, 4)
    U = gauge_field(dims, 0.6, 91)
    op = m.Operator(ctx, U, 0.03, 1.0)
    D = WilsonClover(U, 0.03, 1.0)
    for call, nrhs in enumerate((8, 3)):  # the second call has a smaller input
        x_np = random_spinor(dims, 200 + call, batch=nrhs).reshape(nrhs, -1, 12)
        x = _as_prec(to_gpu(x_np), prec)
        y_ws, yx_ws, yy_ws = op.apply_dot(x, prec=prec)
        y = torch.full_like(x, float("nan"))
        yx = torch.full((nrhs,), complex(float("nan"), 0), dtype=torch.complex128, device=x.device)
        yy = torch.full((nrhs,), float("nan"), dtype=torch.float64, device=x.device)
        op.apply_dot_noalloc(x, y, yx, yy, prec=prec)
        torch.cuda.synchronize()
        assert torch.equal(y, y_ws), (prec, call)
        assert torch.equal(yx, yx_ws) and torch.equal(yy, yy_ws), (prec, call)
        # against the oracle's operator on the same (rounded) input
        xr = from_gpu(_c128(x, prec)).reshape(nrhs, -1)
        want = D.matvec(xr)
        got = from_gpu(_c128(y, prec)).reshape(nrhs, -1)
        assert rel(got, want) < BOUND[prec], (prec, call)
        for r in range(nrhs):
            a = np.vdot(got[r], xr[r])
            b = np.vdot(got[r], got[r]).real
            assert abs(yx[r].item() - a) <= 1e-6 * np.sqrt(b) * np.linalg.norm(xr[r]), (prec, call, r)
            assert abs(yy[r].item() - b) <= 1e-6 * b, (prec, call, r)


def test_noalloc_refuses_shapes_beyond_its_array():
    import torch
    import paper_2509_11424_amd as m
    ctx = m.Context(0)
    dims = (16, 16, 16, 16)
    U = gauge_field(dims, 0.6, 92)
    op = m.Operator(ctx, U, 0.03, 1.0)
    nrhs = 64  # 2 x 64 partials of 16384 blocks: 32 MiB
    assert op.dot_workspace_size(nrhs, "f32") > m.api.NOALLOC_SCRATCH_BYTES
    x = torch.zeros((12, op.V, nrhs), dtype=torch.complex64, device="cuda:0")
    y = torch.empty_like(x)
    yx = torch.empty(nrhs, dtype=torch.complex128, device="cuda:0")
    yy = torch.empty(nrhs, dtype=torch.float64, device="cuda:0")
    with pytest.raises(RuntimeError, match="WORKSPACE"):
        op.apply_dot_noalloc(x, y, yx, yy, prec="f32")
    # 32 rhs fit (8 MiB of partials) and agree with the workspace form
    x = torch.randn((12, op.V, 32), dtype=torch.complex64, device="cuda:0")
    y = torch.empty_like(x)
    yx = torch.empty(32, dtype=torch.complex128, device="cuda:0")
    yy = torch.empty(32, dtype=torch.float64, device="cuda:0")
    op.apply_dot_noalloc(x, y, yx, yy, prec="f32")
    y_ws, yx_ws, yy_ws = op.apply_dot(x, prec="f32")
    torch.cuda.synchronize()
    assert torch.equal(y, y_ws) and torch.equal(yx, yx_ws) and torch.equal(yy, yy_ws)
