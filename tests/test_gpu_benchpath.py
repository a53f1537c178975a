"""Oracle parity of the measured (benchmark) solver path.

The timed estimate runs the mixed-precision form with every production
option on: FP16-storage fine smoothing with the fused lagged-MR step kernel,
nine fine and three coarse smoothing steps, one-step coarse solves, FP32
inner solves of one Arnoldi cycle stopped at a residual drop of 6e-3 (one
classical Gram-Schmidt pass per step), BF16-MFMA coarse operators, FP16 P,
coarse-grid corrections captured into HIP graphs and replayed, autotuned
launch shapes, and uneven per-level batches with ragged tails.  Here the
same settings run on a three-level 8 x 16 x 8 x 4 lattice on which the fused
step kernel applies at every batch size used, solved to the parity tolerance
1e-12, and the per-probe values of every orthogonal tr(D^-1) term (Sec. 3) are
compared with the FP64 oracle's (1e-8 relative, differences X = a - b
against |a| + |b|).  The same settings also solve single batches on every
level against the oracle's solutions.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from gpu_common import to_gpu, from_gpu, rel  # noqa: E402
from lattice_inputs import gauge_field  # noqa: E402

DIMS = (8, 16, 8, 4)
BLOCKS = [(2, 2, 2, 2), (2, 2, 2, 1)]
NTV = [8, 8]
NPROBE = [3, 6, 12]   # probe groups: fine, middle, coarsest
BATCH = [2, 4, 8]     # every group ends in a ragged batch (2+1, 4+2, 8+4)


def bench_solve_desc(m, tol=1e-12):
    return m.solve_desc(tol=tol, kind="mg_mixed", smooth=9, smooth_coarse=3, coarse_iters=1, inner_tol=6e-3,
                        maxiter=5000, coarse_bf16=True, smoother_f16=True, graphs=True)


@pytest.fixture(scope="module")
def bp():
    import torch
    import paper_2509_11424_amd as m
    from oracle.dirac import WilsonClover
    from oracle.multigrid import Hierarchy
    from oracle.solve import level_solver

    class P:
        pass

    p = P()
    p.stream = torch.cuda.Stream(device=0)  # graph capture needs a non-default stream
    p.ctx = m.Context(0, stream=p.stream.cuda_stream)
    p.U = gauge_field(DIMS, 0.6, 81)
    p.op = m.Operator(p.ctx, p.U, 0.05, 1.0)
    p.h = m.Hierarchy(p.op, BLOCKS, NTV, seed=82, max_nrhs=BATCH[0], max_nrhs_level=BATCH, restart=12, mixed=1)
    p.stream.synchronize()
    p.D = WilsonClover(p.U, 0.05, 1.0)
    p.oh = Hierarchy(p.D, BLOCKS, NTV, seed=82)
    p.solvers = [level_solver(o) for o in p.oh.ops]
    return p


def test_fused_step_applies_to_every_fine_batch(bp):
    for nrhs in (1, 2):
        assert bp.op.step_fusable(nrhs), nrhs


def _orthogonal_parts(p, seed, nprobe=NPROBE):
    """Oracle per-probe values of O_0, O_1, F_0, F_1, coarsest, with the
    magnitude |a| + |b| of each difference term X = a - b."""
    from oracle import estimators as E
    from oracle.philox import z4_vector, stream_id, KIND_F
    vals, scales = [], []
    for l in range(2):
        X = E.O_samples(p.oh, p.solvers, l, seed, nprobe[l])
        vals.append(X)
        scales.append(np.abs(X))
    for l in range(2):
        X = E.F_samples(p.oh, p.solvers, l, seed, nprobe[l])
        tr = p.oh.transfers[l]
        sc = np.zeros(nprobe[l])
        for k in range(nprobe[l]):
            x = z4_vector(p.oh.ops[l + 1].n, seed, stream_id(l, KIND_F), k)
            px = tr.prolong(x)
            sc[k] = abs(np.vdot(px, p.solvers[l](px))) + abs(np.vdot(x, p.solvers[l + 1](x)))
        vals.append(X)
        scales.append(sc)
    X = E.coarsest_samples(p.oh, p.solvers, seed, nprobe[2])
    vals.append(X)
    scales.append(np.abs(X))
    return vals, scales


def test_bench_settings_estimate_matches_oracle(bp):
    """Two estimates with the benchmark's settings (the first captures the
    coarse-grid corrections, the second replays them) against the oracle,
    probe by probe; the fused FP16 step kernel must have run."""
    import paper_2509_11424_amd as m
    p = bp
    seed = 83
    want, scale = _orthogonal_parts(p, seed)
    sd = bench_solve_desc(m)
    p.ctx.autotune(True)
    p.ctx.profile(True)
    p.ctx.profile_reset()
    try:
        runs = [p.h.estimate("trace", "orthogonal", NPROBE, seed=seed, batch=BATCH, solve=sd) for _ in range(2)]
        steps = p.ctx.profile_query("dslash_step")["launches"]
    finally:
        p.ctx.profile(False)
        p.ctx.autotune(False)
    p.stream.synchronize()
    assert steps > 0
    for run, res in enumerate(runs):
        assert res["stats"]["max_rel_residual"] <= 1e-12, run
        for q in range(5):
            got = res["samples"][q][:, 0, 0]
            assert got.shape == want[q].shape, (run, q)
            err = np.abs(got - want[q]) / scale[q]
            assert np.all(err <= 1e-8), (run, q, err.max())
        # term statistics are those of the samples (Sec. 4 variance estimator)
        from oracle import estimators as E
        for q in range(5):
            mu, var = E.mean_var(res["samples"][q][:, 0, 0])
            assert abs(res["mean"][q, 0, 0] - mu) <= 1e-12 * abs(mu) + 1e-14
            assert abs(res["var"][q, 0, 0] - var) <= 1e-9 * var + 1e-14


@pytest.mark.parametrize("level", [0, 1, 2])
def test_bench_settings_solves_match_oracle(bp, level):
    """The loose inner solves (6e-3, one Gram-Schmidt pass per Arnoldi step)
    inside FP64 defect correction still converge to the FP64 solution:
    solutions at tol 1e-12 within 1e-9 of the oracle's."""
    import paper_2509_11424_amd as m
    p = bp
    s, d, n = p.h.level_info(level)
    nrhs = BATCH[level] - 1  # ragged against the level's capacity
    rng = np.random.default_rng(84 + level)
    b = rng.standard_normal((nrhs, s, d)) + 1j * rng.standard_normal((nrhs, s, d))
    x, st = p.h.solve(level, to_gpu(b), bench_solve_desc(m))
    p.stream.synchronize()
    assert st["max_rel_residual"] <= 1e-12
    want = np.stack([p.solvers[level](bb) for bb in b.reshape(nrhs, -1)])
    assert rel(from_gpu(x).reshape(nrhs, -1), want) < 1e-9


# More than eight fine right-hand sides: the FP16 smoother stores its vectors
# in column groups (of 8 for 16 rhs, of 4 for 20) and smooths them one group
# at a time (the step kernel runs at the group's rhs count); conversions and
# FP16-input transfers read and write the grouped layout.
CAP16 = [20, 4, 8]
GROUP = {16: 8, 20: 4}


@pytest.fixture(scope="module")
def bp16(bp):
    import paper_2509_11424_amd as m
    h = m.Hierarchy(bp.op, BLOCKS, NTV, seed=82, max_nrhs=CAP16[0], max_nrhs_level=CAP16, restart=12, mixed=1)
    bp.stream.synchronize()
    return h


def _step_keys(p, m):
    rep = p.ctx.tune_report()
    return {n for n in (4, 8, 16, 20) if "dslash_step/%d/%d/%d" % (m.api.PREC["f16"], p.op.V, n) in rep}


@pytest.mark.parametrize("nrhs", [16, 20])
def test_grouped_smoother_solve_matches_oracle(bp, bp16, nrhs):
    """16 and 20 fine right-hand sides with the benchmark's settings:
    solutions at tol 1e-12 within 1e-9 of the oracle's; the step kernel ran
    on the column groups (8 and 4 rhs), never on the whole batch."""
    import paper_2509_11424_amd as m
    p = bp
    s, d, n = bp16.level_info(0)
    rng = np.random.default_rng(86 + nrhs)
    b = rng.standard_normal((nrhs, s, d)) + 1j * rng.standard_normal((nrhs, s, d))
    before = _step_keys(p, m)
    p.ctx.autotune(True)
    try:
        x, st = bp16.solve(0, to_gpu(b), bench_solve_desc(m))
    finally:
        p.ctx.autotune(False)
    p.stream.synchronize()
    assert st["max_rel_residual"] <= 1e-12
    want = np.stack([p.solvers[0](bb) for bb in b.reshape(nrhs, -1)])
    assert rel(from_gpu(x).reshape(nrhs, -1), want) < 1e-9
    keys = _step_keys(p, m) - before
    assert GROUP[nrhs] in _step_keys(p, m) and nrhs not in keys


@pytest.mark.parametrize("nfine", [16, 20])
def test_grouped_smoother_estimate_matches_oracle(bp, bp16, nfine):
    """Estimates with 16 and 20 fine probes in one batch (grouped FP16
    smoother, captured coarse-grid corrections, autotuning) against the oracle
    probe by probe (1e-8 relative, differences against |a| + |b|)."""
    import paper_2509_11424_amd as m
    p = bp
    seed = 87 + nfine
    nprobe = [nfine, 6, 12]
    want, scale = _orthogonal_parts(p, seed, nprobe)
    p.ctx.autotune(True)
    try:
        res = bp16.estimate("trace", "orthogonal", nprobe, seed=seed, batch=[nfine, 4, 8], solve=bench_solve_desc(m))
    finally:
        p.ctx.autotune(False)
    p.stream.synchronize()
    assert res["stats"]["max_rel_residual"] <= 1e-12
    for q in range(5):
        got = res["samples"][q][:, 0, 0]
        assert got.shape == want[q].shape, q
        err = np.abs(got - want[q]) / scale[q]
        assert np.all(err <= 1e-8), (q, err.max())
