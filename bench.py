"""Benchmark of the MG-MLMC hot path on one MI355X.

One step = one orthogonal multigrid multilevel Monte Carlo estimate of
tr(D^-1) (O_l, F_l and coarsest terms, Sec. 3) on the 32^3 x 64 three-level
workload: Z4 probes, projector, transfers, level solves to a relative
residual of 1e-10 (FGMRES + V-cycle, fine dslash, coarse MFMA stencils),
quadratic forms and per-term statistics.  The hierarchy setup (test vectors,
block QR, Galerkin operators) runs once before the timed region and is
reported separately.

value = right-hand sides solved to 1e-10 per second (every level's solves
counted), whole job.  The JSON line also carries the rate of each level alone
(`per_level`: one batch of the level's size solved to 1e-10), the dslash
roofline (HIP events around every dslash launch in the timed region), the
time to reach the target variance of tr(D^-1) in plain FP64 MG and in the
mixed batched form (`time_to_target`, MLMC-optimal probe counts), and the
CPU-oracle baseline (fine-level solve rate of the FP64 oracle on the host's
cores, extrapolated from one operator application per core and the
iteration count of a measured 16^4 solve).

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--config c4|c3|c2]
                  [--form mixed|f64] [--cpu 0|1] [--ttt 0|1] [--learned [--net-widths 4 8 8 4]]
  python bench.py --solve-study --config c3 [--nrhs 12,32,64]   # fine-level RHS/s per form and batch

Kernel micro-benchmarks (used for the profiler runs of single kernels):

  python bench.py --micro dslash|dslash_dot|step --prec f32[,f64,f16] --nrhs 8[,1,...] [--iters 50]
                  [--tune | --variant V]   # autotune the launch shape, or pin variant V
  python bench.py --micro copy [--iters 50]      # plain 1 GiB device copy
  python bench.py --micro coarse --prec bf16 --nrhs 16,100 [--level 1]   # coarse stencil
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "RHS solved/s to 1e-10, dslash HBM GB/s; time-to-target-variance tr(D^-1)"
HBM_PEAK_GBS = 8000.0
# Vector FMA peak without packed FP32 math (the build disables packed FP32):
# 256 CUs x 4 SIMD16 x 16 lanes x 2 flop x 2.4 GHz, the same for FP32 and FP64
VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
DSLASH_FLOP = 1896  # per site and rhs: 8 hops x 168 + clover 552
# the fused smoother step adds r - omega q and x + omega r: 12 complex
# multiply-adds each
FLOP_PER_UNIT = {"dslash_f64": DSLASH_FLOP, "dslash_f32": DSLASH_FLOP, "dslash_f16": DSLASH_FLOP,
                 "dslash_step": DSLASH_FLOP + 2 * 12 * 8}

# HBM traffic of the dominant dslash at nrhs 8 on 32^3 x 64 from two rocprofv3
# --pmc runs, valid only for the kernel sources it was taken with
TRAFFIC_FILES = {
    "dslash_step": os.path.join(ROOT, "profiles", "smoother_step_f16_32x32x32x64_traffic.txt"),
}
PREC_BYTES = {"dslash_f64": 16, "dslash_f32": 8, "dslash_f16": 4, "dslash_step": 4}
# spinor volumes moved per rhs: the dslash reads x and writes y; the fused
# smoother step reads r and writes r', and reads and writes x
SPINOR_VOLUMES = {"dslash_f64": 2, "dslash_f32": 2, "dslash_f16": 2, "dslash_step": 4}
KERNEL_NAMES = {"dslash_f16": "k_dslash<F16, DOT> (fused MR-smoother dslash)",
                "dslash_f32": "k_dslash_rb<F32> (two rhs per thread)", "dslash_f64": "k_dslash<F64>",
                "dslash_step": "k_dslash_march<F16, DOT, MR> (fused FP16 smoother step: dslash, dots, "
                               "r and x updates)"}
N_SITE_VARIANTS_DOT = 2  # site-parallel launch variants of the reducing dslash; plane-marching ones follow
TUNE_PREFIX = {"dslash_step": "dslash_step"}  # tune-table key prefix of each class with recorded counters


def kernel_name(kclass, variants):
    if kclass == "dslash_step":
        return KERNEL_NAMES[kclass]
    if kclass == "dslash_f16" and variants and min(variants.values()) >= N_SITE_VARIANTS_DOT:
        return "k_dslash_march<F16, DOT> (fused MR-smoother dslash, plane-marching)"
    return KERNEL_NAMES[kclass]
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2509_11424_amd", "csrc", f)
                  for f in ("dslash.hip", "fine_dev.h", "fine.h", "common.h")]


def kernel_sources_hash(files=None):
    import hashlib
    h = hashlib.sha256()
    for f in files or KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


# MFMA and HBM counters of the level-1 BF16 coarse stencil of the 32^3 x 64
# workload (8^3 x 16 coarse sites, 48 dof) from rocprofv3 --pmc runs of
# bench.py --micro coarse, with the sources they were taken with
COARSE_MFMA_FILE = os.path.join(ROOT, "profiles", "coarse_bf16_8x8x8x16_d48_mfma.txt")
COARSE_SOURCES = [os.path.join(ROOT, "paper_2509_11424_amd", "csrc", f)
                  for f in ("coarse_mfma.hip", "mg.h", "common.h")]
BF16_MFMA_PEAK_TFLOPS = 2500.0  # dense BF16 matrix-core peak of MI355X


def coarse_mfma_evidence():
    """Matrix-core utilisation and HBM traffic of the level-1 BF16 coarse
    stencil at the rhs counts of its record: executed MFMA flops
    (SQ_INSTS_VALU_MFMA_MOPS_BF16, in units of 512 flop) and useful complex
    block-product flops (8 * 9 * d^2 per site and rhs) per microsecond of the
    autotuned launch, against the dense BF16 peak; calibrated FETCH_SIZE /
    WRITE_SIZE bytes against the algorithmic ones.  None without a record."""
    kv = {}
    try:
        with open(COARSE_MFMA_FILE) as f:
            for line in f:
                if ":" in line and not line.startswith("#") and not line.startswith(" "):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
    except OSError:
        return None
    try:
        sites, d = int(kv["sites"]), int(kv["dof"])
        out = {"kernel": "k_coarse_mfma_bf16 (level-1 coarse stencil, %d sites, %d dof)" % (sites, d),
               "record": os.path.relpath(COARSE_MFMA_FILE, ROOT), "peak_tflops": BF16_MFMA_PEAK_TFLOPS,
               "sources_match": kv.get("kernel_sources_sha256") == kernel_sources_hash(COARSE_SOURCES)}
        fs, ws = float(kv["fetch_scale"]), float(kv["write_scale"])
        for n in [int(v) for v in kv["nrhs"].split()]:
            us = float(kv["avg_us_nrhs%d" % n])
            executed = float(kv["mfma_mops_bf16_nrhs%d" % n]) * 512.0
            useful = 8.0 * 9 * d * d * n * sites
            traffic = (float(kv["fetch_kib_nrhs%d" % n]) * fs + float(kv["write_kib_nrhs%d" % n]) * ws) * 1024.0
            alg = sites * (9.0 * d * d * 4 + 2.0 * d * n * 8)
            out["nrhs%d" % n] = {"variant": int(kv["variant_nrhs%d" % n]), "avg_us": us,
                                 "mfma_tflops_executed": executed / us / 1e6,
                                 "mfma_util": executed / us / 1e6 / BF16_MFMA_PEAK_TFLOPS,
                                 "useful_tflops": useful / us / 1e6,
                                 "hbm_gbps_measured": traffic / us / 1e3,
                                 "hbm_frac_measured": traffic / us / 1e3 / HBM_PEAK_GBS,
                                 "algorithmic_gbps": alg / us / 1e3, "traffic_over_algorithmic": traffic / alg}
        return out
    except (KeyError, ValueError, ZeroDivisionError):
        return None


def dslash_flops(kclass, V, launches, total_bytes):
    """Algorithmic flops of `launches` dslash applications whose algorithmic
    bytes sum to total_bytes (the rhs count of each follows from its bytes)."""
    wc = PREC_BYTES[kclass]
    rhs_total = (total_bytes / V - launches * (36 * wc + 36 * wc)) / (12 * SPINOR_VOLUMES[kclass] * wc)
    return FLOP_PER_UNIT[kclass] * V * rhs_total


def dslash_bytes(kclass, V, nrhs):
    """Algorithmic bytes of one fine dslash (links and clover once, spinors in
    and out), as the library's FineOp::bytes."""
    wc = PREC_BYTES[kclass]
    return V * (36 * wc + 72 * wc / 2 + 12 * SPINOR_VOLUMES[kclass] * wc * nrhs)


def traffic_record(kclass):
    """key: value lines of the counter file of a kernel class ({} if none)."""
    kv = {}
    try:
        with open(TRAFFIC_FILES[kclass]) as f:
            for line in f:
                if ":" in line and not line.startswith("#") and not line.startswith(" "):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
    except (OSError, KeyError):
        pass
    return kv


def rhs_counts(kv):
    """The rhs counts of the timed region's launches that a counter file
    covers, larger first (one or two; 8 and 4 when it does not say)."""
    c = [int(v) for v in kv.get("rhs_counts", "8 4").split()]
    return max(c), min(c)


def measured_traffic(kclass, V, launches, total_bytes, variants=None):
    """Calibrated HBM bytes per launch of the kernel class in the timed region,
    or None.  The counter file holds FETCH_SIZE / WRITE_SIZE per launch at the
    one or two rhs counts the timed region uses on the fine level, taken with
    the launch variants it names; with two, the split of the region's
    launches between them follows from its launch count and algorithmic
    bytes.  None when the counters were taken with other kernel sources or
    launch variants, or the launches do not split into those counts."""
    try:
        kv = traffic_record(kclass)
        if kv.get("kernel_sources_sha256") != kernel_sources_hash():
            return None
        for n, v in (variants or {}).items():
            if "variant_nrhs%d" % n in kv and int(kv["variant_nrhs%d" % n]) != v:
                return None
        hi, lo = rhs_counts(kv)
        fs, ws = float(kv["fetch_scale"]), float(kv["write_scale"])
        t = {n: (float(kv["fetch_kib_nrhs%d" % n]) * fs + float(kv["write_kib_nrhs%d" % n]) * ws) * 1024.0
             for n in (hi, lo)}
        bh, bl = dslash_bytes(kclass, V, hi), dslash_bytes(kclass, V, lo)
        if hi == lo:  # one rhs count: every launch must be of it
            return t[lo] if abs(total_bytes - launches * bl) <= 1e-6 * total_bytes else None
        nh = (total_bytes - launches * bl) / (bh - bl)
        if abs(nh - round(nh)) > 1e-3 * launches or nh < -0.5 or nh > launches + 0.5:
            return None
        nh = int(round(nh))
        return (nh * t[hi] + (launches - nh) * t[lo]) / launches
    except (OSError, KeyError, ValueError, ZeroDivisionError):
        return None


CONFIGS = {
    # 32^3 x 64, csw 1, roughness 0.6, m0 0.02; 4^4 (24 tv) then 2^4 (32 tv);
    # probes 20 / 100 / 400 on the fine / middle / coarsest difference levels
    # batch: rhs per solve batch on each level in the mixed form (all 20
    # fine-level probes of a term at once, 238 GB of workspace, its FP16
    # smoother in five column groups of 4; all 100 middle-level probes of a
    # term at once; 80 on the coarsest); the FP64 form of the time-to-target
    # comparison keeps 8 on the fine level (its FP64 Krylov workspace would
    # need about 245 GB at 16)
    "c4": dict(dims=(32, 32, 32, 64), eps=0.6, m0=0.02, csw=1.0, gseed=14, blocks=[(4, 4, 4, 4), (2, 2, 2, 2)],
               ntv=[24, 32], nprobe=[20, 100, 400], pseed=104, batch=[20, 100, 80], batch_f64=[8, 100, 80],
               aux_fine_batch=8,
               # with --learned: the network's activations at the time-to-target
               # run need the room a fine batch of 16 leaves (198 GB hierarchy)
               batch_learned=[16, 100, 80],
               restart=12,
               name="32^3x64 Wilson-clover (csw 1, roughness 0.6, m0 0.02), 3-level orthogonal MG-MLMC "
                    "tr(D^-1), aggregates 4^4/2^4, N_tv 24/32, probes 20/100/400"),
    # one GPU's share of the paper's J501 lattice (192 x 64^3 split four ways
    # in time) with its four-level aggregation 4^4 / 2^4 / 2^4 (coarse
    # lattices 16^3 x 12, 8^3 x 6, 4^3 x 3); synthetic field of the same
    # family as the 32^3 x 64 workload
    "j501q": dict(dims=(64, 64, 64, 48), eps=0.6, m0=0.02, csw=1.0, gseed=15,
                  blocks=[(4, 4, 4, 4), (2, 2, 2, 2), (2, 2, 2, 2)], ntv=[24, 32, 32], nprobe=[4, 8, 16, 64],
                  pseed=105, batch=[2, 8, 16, 32], batch_f64=[2, 8, 16, 32], restart=8,
                  name="64^3x48 Wilson-clover (csw 1, roughness 0.6, m0 0.02; one quarter of J501's 192x64^3 in "
                       "time), 4-level orthogonal MG-MLMC tr(D^-1), aggregates 4^4/2^4/2^4, N_tv 24/32/32, "
                       "probes 4/8/16/64"),
    "c3": dict(dims=(16, 16, 16, 16), eps=0.6, m0=0.01, csw=1.0, gseed=13, blocks=[(2, 2, 2, 2)], ntv=[12],
               nprobe=[64, 256], pseed=103, batch=[32, 64], restart=16,
               name="16^4 Wilson-clover (csw 1, roughness 0.6, m0 0.01), 2-level orthogonal MG-MLMC tr(D^-1), "
                    "2^4 aggregates, N_tv 12"),
    "c2": dict(dims=(8, 8, 8, 8), eps=0.5, m0=0.05, csw=1.0, gseed=12, blocks=[(2, 2, 2, 2)], ntv=[8],
               nprobe=[50, 200], pseed=102, batch=[25, 64], restart=16,
               name="8^4 Wilson-clover (csw 1, roughness 0.5, m0 0.05), 2-level orthogonal MG-MLMC tr(D^-1), "
                    "2^4 aggregates, N_tv 8, probes 50/200"),
}


def aux_fine_batch(cfg):
    """Fine-level batch of the observables and hierarchy-study legs, whose
    hierarchies hold more fine vectors per rhs than the trace bench's: the
    configuration's own value (8 on the 32^3 x 64 workload), else half the
    trace bench's fine batch."""
    return cfg.get("aux_fine_batch", max(1, cfg["batch"][0] // 2))


def rhs_per_step(nprobe):
    """Solves of one right-hand side per orthogonal estimate: O_l (level l),
    F_l (levels l and l+1), coarsest."""
    L = len(nprobe)
    return sum(3 * nprobe[l] for l in range(L - 1)) + nprobe[L - 1]


# ------------------------------------------------------------ CPU baseline

CPU_WORKERS_MAX = 16  # host cores of one GPU's share on the GPU machine


def _cpu_apply_worker(D, seed, conn):
    """One FP64 oracle application in a forked worker (single-threaded BLAS)."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):
        x = np.random.default_rng(seed).standard_normal(D.n) + 0j
        conn.send(time.time())
        D.matvec(x)
        conn.send(time.time())
    conn.close()


def cpu_baseline(cfg, U, out_path):
    """The FP64 numpy oracle on the host, on a bounded sample of the workload.

    * single thread (BLAS limited to one thread with threadpoolctl): one
      Wilson-clover application on the workload's lattice, and one GMRES(50)
      solve of a Z4 right-hand side to a true relative residual of 1e-10 on
      the 16^4 lattice of the same ensemble family (m0 0.01, roughness 0.6),
      whose iteration count extrapolates the fine-level solve rate of the
      workload (labelled extrapolated);
    * all cores: the same application in W forked single-threaded workers at
      once (W = min(16, cores)), i.e. independent probes run side by side.
    Writes a JSON dict to out_path."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    res = {}
    try:
        from oracle.dirac import WilsonClover
        from oracle.solve import gmres
        from oracle.philox import z4_vector
        ncpu = os.cpu_count() or 1
        workers = max(1, min(CPU_WORKERS_MAX, ncpu))
        with threadpool_limits(1):
            t0 = time.time()
            D = WilsonClover(U, cfg["m0"], cfg["csw"])
            t_build = time.time() - t0
            x = np.random.default_rng(0).standard_normal(D.n) + 0j
            t0 = time.time()
            D.matvec(x)
            t_apply = time.time() - t0
            del x
        # all cores: W workers, one application each, started together
        import multiprocessing as mp
        ctxm = mp.get_context("fork")
        pipes, procs = [], []
        for w in range(workers):
            a, b = ctxm.Pipe(duplex=False)
            pr = ctxm.Process(target=_cpu_apply_worker, args=(D, 10 + w, b))
            pr.start()
            pipes.append(a)
            procs.append(pr)
        starts = [p.recv() for p in pipes]
        ends = [p.recv() for p in pipes]
        for pr in procs:
            pr.join()
        t_all = max(ends) - min(starts)
        del D
        # measured solve at 16^4 (single thread)
        from lattice_inputs import gauge_field
        with threadpool_limits(1):
            U3 = gauge_field((16, 16, 16, 16), 0.6, 13)
            D3 = WilsonClover(U3, 0.01, 1.0)
            count = [0]

            def mv(v):
                count[0] += 1
                return D3.matvec(v)

            b = z4_vector(D3.n, 103, 0, 0)
            t0 = time.time()
            gmres(mv, b, tol=1e-10, restart=50)
            t_solve3 = time.time() - t0
        iters = count[0]
        lat = "x".join(map(str, cfg["dims"]))
        single = 1.0 / (t_apply * iters)
        allcore = workers / (t_all * iters)
        res = {"value": allcore, "unit": "RHS/s", "cores": workers, "kind": "oracle",
               "sample": "numpy FP64 oracle, fine-level RHS/s on %s, extrapolated: %d single-threaded workers "
                         "each apply D once side by side (%.2f s wall), times the %d GMRES(50) applications the "
                         "oracle needed for one Z4 right-hand side to 1e-10 on 16^4 (measured, %.1f s); host "
                         "reports %d cores" % (lat, workers, t_all, iters, t_solve3, ncpu),
               "extrapolated": True, "nproc": ncpu,
               "single_thread": {"value": single, "unit": "RHS/s", "cores": 1, "t_apply_s": t_apply,
                                 "t_build_s": t_build},
               "all_cores": {"value": allcore, "workers": workers, "t_apply_wall_s": t_all},
               "solve_16x16x16x16": {"seconds": t_solve3, "applications": iters, "tol": 1e-10,
                                     "rhs_per_s": 1.0 / t_solve3, "cores": 1}}
    except Exception as e:  # reported, never fatal for the GPU leg
        res = {"error": repr(e)}
    with open(out_path, "w") as f:
        json.dump(res, f)


# ------------------------------------------------------------------- GPU

def progress(msg):
    """One progress line on stderr (the JSON result stays alone on stdout)."""
    print("[bench] " + msg, file=sys.stderr, flush=True)


def run_batches(cfg, form, learned, batch=None):
    """Per-level batches of the timed run: the FP64 form's own (its Krylov
    workspace), with --learned the ones its measurement used, else the
    configuration's; an explicit --batch wins."""
    if batch:
        return list(batch)
    if form == "f64" and "batch_f64" in cfg:
        return list(cfg["batch_f64"])
    if learned and "batch_learned" in cfg:
        return list(cfg["batch_learned"])
    return list(cfg["batch"])


def run(args):
    import numpy as np
    cfg = dict(CONFIGS[args.config])
    cfg["batch"] = run_batches(cfg, args.form, args.learned, args.batch)
    from lattice_inputs import gauge_field
    t0 = time.time()
    U = gauge_field(cfg["dims"], cfg["eps"], cfg["gseed"])
    t_gauge = time.time() - t0
    progress("gauge field %s generated in %.1f s" % ("x".join(map(str, cfg["dims"])), t_gauge))
    cpu_pid = None
    cpu_out = os.path.join("/tmp", "mgm_cpu_baseline_%d.json" % os.getpid())
    if args.cpu:
        # fork before any GPU call: the child only runs numpy (BLAS threads
        # limited inside it with threadpoolctl)
        cpu_pid = os.fork()
        if cpu_pid == 0:
            try:
                cpu_baseline(cfg, U, cpu_out)
            finally:
                os._exit(0)
    import torch
    import paper_2509_11424_amd as m
    # a dedicated stream (default priority): torch work and the library share
    # it, and the coarse-grid corrections can be captured into HIP graphs
    stream = torch.cuda.Stream(device=0)
    with torch.cuda.stream(stream):
        _run_gpu(args, cfg, U, t_gauge, cpu_pid, cpu_out, m, torch)


def roofline(ds, V, q, achieved_gbs, avg_ms, bytes_launch, variants, traffic):
    """Roofline of the dominant dslash against whichever roof is tighter for
    its algorithmic counts: FP32/FP64 vector FMA (unpacked) or HBM."""
    flops_launch = dslash_flops(ds, V, q["launches"], q["bytes"]) / max(q["launches"], 1)
    tflops = flops_launch / (avg_ms * 1e-3) / 1e12 if q["launches"] else 0.0
    t_alu = flops_launch / (VALU_PEAK_TFLOPS * 1e12)
    t_hbm = bytes_launch / (HBM_PEAK_GBS * 1e9)
    hbm = {"achieved": achieved_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved_gbs / HBM_PEAK_GBS}
    alu = {"achieved": tflops, "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": tflops / VALU_PEAK_TFLOPS}
    main, other, bound = (alu, hbm, "alu") if t_alu > t_hbm else (hbm, alu, "hbm")
    out = {"bound": bound}
    out.update(main)
    out.update({"traffic": traffic, "kernel": kernel_name(ds, variants), "launch_variants": variants,
                "avg_launch_ms": avg_ms, "launches": q["launches"], "bytes_per_launch": bytes_launch,
                "flop_per_launch": flops_launch, "other_roof": dict(other, bound="hbm" if bound == "alu" else "alu"),
                "peak_note": "alu peak = unpacked vector FMA (packed FP32 is disabled in the build; "
                             "the packed FP32 figure is 157.3 TFLOP/s)"})
    return out


def _run_gpu(args, cfg, U, t_gauge, cpu_pid, cpu_out, m, torch):
    ctx = m.Context(0)
    op = m.Operator(ctx, U, cfg["m0"], cfg["csw"])
    L = len(cfg["blocks"]) + 1
    mixed = 1 if args.form == "mixed" else 0
    t0 = time.time()
    h = m.Hierarchy(op, cfg["blocks"], cfg["ntv"], seed=cfg["pseed"] + 1000, max_nrhs=cfg["batch"][0],
                    max_nrhs_level=cfg["batch"], restart=cfg["restart"], mixed=mixed)
    torch.cuda.synchronize()
    t_setup = time.time() - t0
    progress("hierarchy built in %.1f s" % t_setup)
    kind = "mg_mixed" if mixed else "mg"
    # mixed form: FP16-storage fine smoother, BF16 MFMA coarse operators,
    # autotuned launch shapes and graph-captured coarse-grid corrections
    # smoothing 9 / 3 (mixed form; 6 / 2 for FP64) on the fine / coarser levels, one
    # coarse-solve step and (mixed form) FP32 inner solves that reduce the
    # residual by 6e-3 per FP64 defect-correction cycle: the fastest settings
    # measured for each form
    sd = m.solve_desc(tol=1e-10, kind=kind, smooth=args.smooth, smooth_coarse=args.smooth_coarse,
                      coarse_iters=args.coarse_iters, inner_tol=args.inner_tol,
                      maxiter=5000, coarse_bf16=True, smoother_f16=True, graphs=bool(mixed))
    # launch-shape keys of the kernel classes with recorded HBM counters
    pin_keys = {kc: {n: "%s/%d/%d/%d" % (TUNE_PREFIX[kc], m.api.PREC["f16"], op.V, n)
                     for n in rhs_counts(traffic_record(kc))} for kc in TUNE_PREFIX}
    if mixed:
        # on the workload the HBM counters were recorded on, the smoother
        # kernels keep the launch shapes of the record (the fastest measured);
        # everything else is tuned
        for kc, keys in (pin_keys.items() if args.config == "c4" else ()):
            rec = traffic_record(kc)
            for n, key in keys.items():
                if "variant_nrhs%d" % n in rec:
                    ctx.tune_set(key, int(rec["variant_nrhs%d" % n]))
        ctx.autotune(True)
    batch = cfg["batch"]

    def step(first):
        return h.estimate("trace", "orthogonal", cfg["nprobe"], seed=cfg["pseed"], batch=batch,
                          first_probe=first, solve=sd, samples=False)

    for w in range(args.warmup):
        step(0)
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.profile_reset()
    results = []
    torch.cuda.synchronize()
    t0 = time.time()
    for k in range(args.steps):
        results.append(step((k + 1) * 1000))
    torch.cuda.synchronize()
    dt = time.time() - t0
    prof = {c: ctx.profile_query(c) for c in ("dslash_f64", "dslash_f32", "dslash_f16", "dslash_step",
                                               "coarse_f64", "coarse_f32", "coarse_bf16", "transfer")}
    ctx.profile(False)
    nrhs_step = rhs_per_step(cfg["nprobe"])
    value = nrhs_step * args.steps / dt
    # dominant kernel: the dslash precision class with the most time
    ds = max(("dslash_f64", "dslash_f32", "dslash_f16", "dslash_step"), key=lambda k: prof[k]["ms"])
    q = prof[ds]
    rep = ctx.tune_report()
    # launch variants the dominant class ran with, per rhs count (pinned or tuned)
    pref = "%s/%d/%d/" % (TUNE_PREFIX.get(ds, ""), m.api.PREC["f16"], op.V)
    variants = {int(k[len(pref):]): v[0] for k, v in rep.items() if ds in TUNE_PREFIX and k.startswith(pref)}
    avg_ms = q["ms"] / max(q["launches"], 1)
    bytes_launch = q["bytes"] / max(q["launches"], 1)
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9 if q["launches"] else 0.0
    line = {
        "metric": METRIC, "value": value, "unit": "RHS/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+bf16 (f64 defect correction)" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "lattice": "x".join(map(str, cfg["dims"])), "levels": L,
                   "probes": cfg["nprobe"], "batch": batch, "tol": 1e-10, "form": args.form,
                   "smoothing": [sd.smooth, sd.smooth_coarse], "coarse_iters": sd.coarse_iters,
                   "inner_tol": sd.inner_tol},
        "roofline": roofline(ds, op.V, q, achieved, avg_ms, bytes_launch, variants,
                             measured_traffic(ds, op.V, q["launches"], q["bytes"], variants)
                             if args.config == "c4" else None),
        "hierarchy_workspace_gb": h.ws.numel() / 1e9,
        "setup_s": t_setup, "gauge_gen_s": t_gauge, "rhs_per_step": nrhs_step,
        "solver_iterations_per_step": results[-1]["stats"]["iterations"],
        "estimate": {"tr_Dinv": [results[-1]["total_mean"][0, 0].real, results[-1]["total_mean"][0, 0].imag],
                     "var_of_mean": float(results[-1]["total_var"][0, 0]),
                     "term_var": [float(v) for v in results[-1]["var"][:, 0, 0]],
                     "term_cost_s": [float(c) for c in results[-1]["cost_s"]]},
        "kernels": {k: {"launches": v["launches"], "ms": v["ms"],
                        "GBps": (v["bytes"] / v["ms"] / 1e6) if v["ms"] > 0 else 0.0} for k, v in prof.items()},
        "kernels_note": "HIP-event statistics of eagerly launched kernels; launches replayed from the captured "
                        "coarse-grid-correction graphs are not timed per class",
        "tuned_shapes": len(ctx.tune_report()) if mixed else 0,
        "coarse_mfma": coarse_mfma_evidence(),
    }
    progress("timed steps done: %.1f RHS/s" % value)
    line["per_level"] = per_level_rates(m, ctx, h, cfg, sd, batch, torch)
    progress("per-level rates done")
    weights = None
    if args.learned or args.ttt:
        del h, results
        torch.cuda.empty_cache()
    if args.learned:
        line["learned"], weights = learned_form(m, ctx, args, torch)
    if args.ttt:

        def make_mixed():
            return m.Hierarchy(op, cfg["blocks"], cfg["ntv"], seed=cfg["pseed"] + 1000, max_nrhs=cfg["batch"][0],
                               max_nrhs_level=cfg["batch"], restart=cfg["restart"], mixed=1)

        line["time_to_target"] = time_to_target(m, ctx, op, cfg, make_mixed, sd, args, weights)
        progress("time to target done")
    if cpu_pid:
        os.waitpid(cpu_pid, 0)
        try:
            with open(cpu_out) as f:
                line["cpu_baseline"] = json.load(f)
            os.remove(cpu_out)
        except Exception as e:
            line["cpu_baseline"] = {"error": repr(e)}
    print(json.dumps(line), flush=True)


def micro_coarse(args, cfg, m, ctx, op, g, torch):
    """Times the coarse stencil of level `--level` (default 1) of the
    workload's mixed hierarchy in precision bf16 / f32 / f64 (HIP events on
    the library's stream, autotuned tiles), for each rhs count."""
    nmax = max(int(v) for v in args.nrhs.split(","))
    caps = [1] + [nmax] * (len(cfg["blocks"]))
    h = m.Hierarchy(op, cfg["blocks"], cfg["ntv"], seed=cfg["pseed"] + 1000, max_nrhs=1, max_nrhs_level=caps,
                    restart=2, mixed=2)
    lvl = args.level
    s_, d_, _ = h.level_info(lvl)
    kc = {"bf16": "coarse_bf16", "f32": "coarse_f32", "f64": "coarse_f64"}
    for prec in args.prec.split(","):
        for nrhs in [int(v) for v in args.nrhs.split(",")]:
            dt = torch.complex128 if prec == "f64" else torch.complex64
            x = torch.randn((d_, s_, nrhs), generator=g, device="cuda:0", dtype=dt)
            ctx.autotune(True)
            for _ in range(3):
                h.apply_prec(lvl, x, prec)
            ctx.autotune(False)
            torch.cuda.synchronize()
            ctx.profile(True)
            ctx.profile_reset()
            for _ in range(args.iters):
                h.apply_prec(lvl, x, prec)
            torch.cuda.synchronize()
            q = ctx.profile_query(kc[prec])
            ctx.profile(False)
            ms = q["ms"] / q["launches"]
            bl = q["bytes"] / q["launches"]
            flop = 8.0 * 9 * d_ * d_ * nrhs * s_  # complex multiply-adds of the nine blocks
            print(json.dumps({"micro": "coarse", "prec": prec, "level": lvl, "sites": s_, "dof": d_, "nrhs": nrhs,
                              "launches": q["launches"], "avg_ms": ms, "bytes_per_launch": bl,
                              "GBps": bl / ms / 1e6, "TFLOPs": flop / ms / 1e9}), flush=True)
            del x


def observables(args):
    """The configuration's observables with the timed form's solver (mixed,
    FP16 smoother, BF16 coarse stencils, graphs): the connected
    pseudoscalar correlator C(t) for every t with the orthogonal, oblique and
    plain decompositions (Sec. 1.1, eq. connected-G; Sec. 4.1), and the
    disconnected loops tr(Gamma D^-1) per time slice for the six Gamma with
    the orthogonal and plain decompositions (Sec. 4.3).  One JSON line per
    (observable, decomposition): per-t means and variances of the mean, the
    per-term variance summed over t, solver seconds per term and wall time.
    Plain runs as many fine-level probes as the finest difference level."""
    import numpy as np
    cfg = dict(CONFIGS[args.config])
    if args.batch:
        cfg["batch"] = list(args.batch)
    from lattice_inputs import gauge_field
    U = gauge_field(cfg["dims"], cfg["eps"], cfg["gseed"])
    import torch
    import paper_2509_11424_amd as m
    stream = torch.cuda.Stream(device=0)
    with torch.cuda.stream(stream):
        ctx = m.Context(0)
        op = m.Operator(ctx, U, cfg["m0"], cfg["csw"])
        L = len(cfg["blocks"]) + 1
        # a smaller fine batch than the trace bench's: the fine-level term
        # vectors of correlators and loops take (4L - 3) fine vectors per rhs
        batch = [aux_fine_batch(cfg)] + list(cfg["batch"][1:])
        h = m.Hierarchy(op, cfg["blocks"], cfg["ntv"], seed=cfg["pseed"] + 1000, max_nrhs=batch[0],
                        max_nrhs_level=batch, restart=cfg["restart"], mixed=1, with_corr=True)
        sd = m.solve_desc(tol=1e-10, kind="mg_mixed", smooth=args.smooth, smooth_coarse=args.smooth_coarse,
                          coarse_iters=args.coarse_iters, inner_tol=args.inner_tol, maxiter=5000,
                          coarse_bf16=True, smoother_f16=True, graphs=True)
        ctx.autotune(True)
        T = cfg["dims"][3]
        nprobe = list(args.obs_probes) if args.obs_probes else list(cfg["nprobe"])
        for obs, decs in (("corr", ("orthogonal", "oblique", "plain")), ("loops", ("orthogonal", "plain"))):
            for dec in decs:
                npr = nprobe if dec != "plain" else [nprobe[0]] + [0] * (L - 1)
                print(json.dumps({"start": obs, "decomposition": dec, "nprobe": npr}), flush=True)
                torch.cuda.synchronize()
                t0 = time.time()
                # the sources of every probe group of correlators and loops
                # live on the fine lattice: batches of the fine level's size
                r = h.estimate(obs, dec, npr, seed=cfg["pseed"] + 21, batch=batch[0], solve=sd, samples=False)
                torch.cuda.synchronize()
                dt = time.time() - t0
                mean, var = r["total_mean"], r["total_var"]
                line = {"observable": obs, "decomposition": dec, "workload": cfg["name"], "T": T,
                        "nprobe": npr, "batch": batch, "seconds": dt,
                        "max_rel_residual": r["stats"]["max_rel_residual"],
                        "term_var_sum_t": [[float(v) for v in r["var"][q].sum(axis=1)] for q in range(len(r["n"]))],
                        "term_cost_s": [float(c) for c in r["cost_s"]], "term_n": [int(n) for n in r["n"]]}
                if obs == "corr":
                    line["C_t"] = [float(v) for v in mean[0].real]
                    line["var_of_mean_t"] = [float(v) for v in var[0]]
                else:
                    line["gammas"] = ["1", "gamma5", "gamma1", "gamma2", "gamma3", "gamma4"]
                    line["loop_t_re"] = [[float(v) for v in mean[g].real] for g in range(mean.shape[0])]
                    line["loop_t_im"] = [[float(v) for v in mean[g].imag] for g in range(mean.shape[0])]
                    line["var_of_mean_t"] = [[float(v) for v in var[g]] for g in range(var.shape[0])]
                print(json.dumps(line), flush=True)
        del h
        torch.cuda.empty_cache()


def hierarchy_study(args):
    """Variance per term against setup cost for richer hierarchies (Sec. 5:
    more test vectors, test vectors with small eigen-residuals).  For each
    variant -- the configuration's N_tv, N_tv 64 on the first transfer, and
    the configuration's N_tv with the fine test vectors refined to
    eigen-residual 1e-4 -- one JSON line: setup and refinement seconds, the
    orthogonal estimate's per-term variance and solver cost at the
    configured probe counts with the timed form's solver, and the
    figure of merit (sum_q sqrt(var_q cost_q))^2, the MLMC cost of any fixed
    target variance up to a common factor (Sec. 2.2, eq. MLMC-Nl)."""
    import numpy as np
    cfg = dict(CONFIGS[args.config])
    from lattice_inputs import gauge_field
    U = gauge_field(cfg["dims"], cfg["eps"], cfg["gseed"])
    import torch
    import paper_2509_11424_amd as m
    stream = torch.cuda.Stream(device=0)
    with torch.cuda.stream(stream):
        ctx = m.Context(0)
        op = m.Operator(ctx, U, cfg["m0"], cfg["csw"])
        # a smaller fine batch than the trace bench's: room for 64 test
        # vectors and for the refinement's block vectors
        batch = [aux_fine_batch(cfg)] + list(cfg["batch"][1:])
        sd = m.solve_desc(tol=1e-10, kind="mg_mixed", smooth=args.smooth, smooth_coarse=args.smooth_coarse,
                          coarse_iters=args.coarse_iters, inner_tol=args.inner_tol, maxiter=5000,
                          coarse_bf16=True, smoother_f16=True, graphs=True)
        ctx.autotune(True)
        variants = [("default", list(cfg["ntv"]), False), ("ntv64", [64] + list(cfg["ntv"][1:]), False),
                    ("refined", list(cfg["ntv"]), True)]
        for name, ntv, refine in variants:
            print(json.dumps({"start": name, "ntv": ntv}), flush=True)
            torch.cuda.synchronize()
            t0 = time.time()
            h = m.Hierarchy(op, cfg["blocks"], ntv, seed=cfg["pseed"] + 1000, max_nrhs=batch[0],
                            max_nrhs_level=batch, restart=cfg["restart"], mixed=1)
            torch.cuda.synchronize()
            line = {"study": "hierarchy", "variant": name, "workload": cfg["name"], "ntv": ntv,
                    "setup_s": time.time() - t0, "hierarchy_workspace_gb": h.ws.numel() / 1e9}
            if refine:
                rsd = m.solve_desc(tol=1e-6, kind="mg_mixed", smooth=args.smooth, smooth_coarse=args.smooth_coarse,
                                   coarse_iters=args.coarse_iters, inner_tol=args.inner_tol, maxiter=5000,
                                   coarse_bf16=True, smoother_f16=True, graphs=True)
                st = h.refine(max_iters=12, eig_tol=1e-4, power_tol=1e-6, batch=batch[0], solve=rsd)
                line["refine"] = {k: st[k] for k in ("steps", "converged", "max_rho_start", "max_rho", "seconds")}
            r = h.estimate("trace", "orthogonal", cfg["nprobe"], seed=cfg["pseed"] + 7, batch=batch, solve=sd,
                           samples=False)
            torch.cuda.synchronize()
            t1 = time.time()
            r = h.estimate("trace", "orthogonal", cfg["nprobe"], seed=cfg["pseed"] + 7, batch=batch, solve=sd,
                           samples=False)
            torch.cuda.synchronize()
            var, cost = r["var"][:, 0, 0], r["cost_s"]
            line.update({"estimate_s": time.time() - t1, "term_var": [float(v) for v in var],
                         "term_cost_s": [float(c) for c in cost], "term_n": [int(n) for n in r["n"]],
                         "total_var_of_mean": float(r["total_var"][0, 0]),
                         "mlmc_merit": float(np.sum(np.sqrt(np.maximum(var, 0) * cost)) ** 2),
                         "iterations": r["stats"]["iterations"]})
            print(json.dumps(line), flush=True)
            del h, r
            torch.cuda.empty_cache()


def _cpu_mlmc_worker(args_conn):
    """One forked worker of the host MG-MLMC run: its share of the probes of
    every orthogonal term, solved by the oracle (single-threaded BLAS)."""
    (oh, seed, ranges, conn) = args_conn
    from threadpoolctl import threadpool_limits
    from oracle import estimators as E
    from oracle.solve import level_solver
    with threadpool_limits(1):
        t0 = time.time()
        solvers = [level_solver(o, tol=1e-10) for o in oh.ops]
        out = {"O": E.O_samples(oh, solvers, 0, seed, ranges[0][1], first=ranges[0][0]).tolist(),
               "F": E.F_samples(oh, solvers, 0, seed, ranges[1][1], first=ranges[1][0]).tolist(),
               "C": E.coarsest_samples(oh, solvers, seed, ranges[2][1], first=ranges[2][0]).tolist()}
        out["seconds"] = time.time() - t0
    conn.send(json.dumps({k: ([[v.real, v.imag] for v in val] if isinstance(val, list) else val)
                          for k, val in out.items()}))
    conn.close()


def cpu_study(args):
    """The FP64 oracle on the host cores at the small workloads (no GPU): per
    workload one Wilson(-clover) application and one GMRES(50) solve of a Z4
    right-hand side to a true relative residual of 1e-10, single-threaded;
    and the whole two-level orthogonal MG-MLMC tr(D^-1) estimate on 8^4 at
    50 / 200 probes (hierarchy single-threaded, the probes split over forked
    single-threaded workers).  One JSON line per measurement."""
    import numpy as np
    import multiprocessing as mp
    from threadpoolctl import threadpool_limits
    from lattice_inputs import gauge_field
    from oracle.dirac import WilsonClover
    from oracle.solve import gmres
    from oracle.philox import z4_vector
    from oracle.multigrid import Hierarchy
    ncpu = os.cpu_count() or 1
    workers = max(1, min(CPU_WORKERS_MAX, ncpu))
    cases = [("4^4 Wilson (m0 0.2)", (4, 4, 4, 4), 0.3, 11, 0.2, 0.0),
             ("8^4 Wilson-clover (m0 0.05, roughness 0.5)", (8, 8, 8, 8), 0.5, 12, 0.05, 1.0),
             ("16^4 Wilson-clover (m0 0.01, roughness 0.6)", (16, 16, 16, 16), 0.6, 13, 0.01, 1.0)]
    for name, dims, eps, gseed, m0, csw in cases:
        with threadpool_limits(1):
            U = gauge_field(dims, eps, gseed)
            t0 = time.time()
            D = WilsonClover(U, m0, csw)
            t_build = time.time() - t0
            x = np.random.default_rng(0).standard_normal(D.n) + 0j
            t0 = time.time()
            D.matvec(x)
            t_apply = time.time() - t0
            cnt = [0]

            def mv(v):
                cnt[0] += 1
                return D.matvec(v)

            b = z4_vector(D.n, 7, 0, 0)
            t0 = time.time()
            xs = gmres(mv, b, tol=1e-10, restart=50)
            t_solve = time.time() - t0
            res = float(np.linalg.norm(b - D.matvec(xs)) / np.linalg.norm(b))
        print(json.dumps({"cpu_study": "apply_and_solve", "workload": name, "sites": int(np.prod(dims)),
                          "cores": 1, "build_s": t_build, "apply_s": t_apply,
                          "apply_GBps": 1536.0 * np.prod(dims) / t_apply / 1e9,
                          "solve_s": t_solve, "applications": cnt[0], "rel_residual": res}), flush=True)
    # whole 8^4 two-level orthogonal estimate (50 / 200 probes)
    cfg = CONFIGS["c2"]
    with threadpool_limits(1):
        U = gauge_field(cfg["dims"], cfg["eps"], cfg["gseed"])
        t_all = time.time()
        D = WilsonClover(U, cfg["m0"], cfg["csw"])
        t0 = time.time()
        oh = Hierarchy(D, cfg["blocks"], cfg["ntv"], seed=cfg["pseed"] + 1000)
        t_setup = time.time() - t0
    n0, n1 = cfg["nprobe"]

    def split(n, w):
        base, extra = divmod(n, w)
        out, first = [], 0
        for i in range(w):
            k = base + (1 if i < extra else 0)
            out.append((first, k))
            first += k
        return out

    so, sf, sc = split(n0, workers), split(n0, workers), split(n1, workers)
    ctxm = mp.get_context("fork")
    pipes, procs = [], []
    t0 = time.time()
    for w in range(workers):
        a, bconn = ctxm.Pipe(duplex=False)
        pr = ctxm.Process(target=_cpu_mlmc_worker, args=((oh, cfg["pseed"], (so[w], sf[w], sc[w]), bconn),))
        pr.start()
        pipes.append(a)
        procs.append(pr)
    parts = [json.loads(pp.recv()) for pp in pipes]
    for pr in procs:
        pr.join()
    t_probes = time.time() - t0
    samples = {k: np.array([complex(*v) for p_ in parts for v in p_[k]]) for k in ("O", "F", "C")}
    var = {k: float(np.sum(np.abs(v - v.mean()) ** 2) / (len(v) - 1)) for k, v in samples.items()}
    total = sum(complex(v.mean()) for v in samples.values())
    total_var = sum(var[k] / len(samples[k]) for k in samples)
    print(json.dumps({"cpu_study": "mlmc_8x8x8x8", "workload": cfg["name"], "cores": workers,
                      "setup_s_single_thread": t_setup, "probes_s_wall": t_probes,
                      "worker_seconds_sum": sum(p_["seconds"] for p_ in parts),
                      "total_s": time.time() - t_all, "rhs_solved": n0 + 2 * n0 + n1,
                      "tr_Dinv": [total.real, total.imag], "var_of_mean": total_var, "term_var": var}),
          flush=True)


def solve_study(args):
    """RHS solved per second to 1e-10 on the fine level over batch size and
    form: plain FP64 multigrid, the mixed form without captured coarse-grid
    corrections and the mixed form with them (each with the settings the
    time-to-target comparison uses for it; autotuned launch shapes in the
    mixed forms), hierarchy setup timed apart.  One JSON line per (form,
    batch) of Z4 right-hand sides: seconds of one solve after an untimed solve
    of the same batch, iterations, and each right-hand side's true residual
    |b - D x| / |b| recomputed with the FP64 operator; only the right-hand
    sides at or below 1e-10 are counted in the rate."""
    cfg = dict(CONFIGS[args.config])
    from lattice_inputs import gauge_field
    U = gauge_field(cfg["dims"], cfg["eps"], cfg["gseed"])
    import torch
    import paper_2509_11424_amd as m
    sizes = [int(v) for v in (args.nrhs or "12,32,64").split(",")]
    stream = torch.cuda.Stream(device=0)
    with torch.cuda.stream(stream):
        ctx = m.Context(0)
        op = m.Operator(ctx, U, cfg["m0"], cfg["csw"])
        for mixed in (0, 1):
            torch.cuda.synchronize()
            t0 = time.time()
            h = m.Hierarchy(op, cfg["blocks"], cfg["ntv"], seed=cfg["pseed"] + 1000, max_nrhs=max(sizes),
                            restart=cfg["restart"], mixed=mixed)
            torch.cuda.synchronize()
            setup = time.time() - t0
            print(json.dumps({"study": "solve", "workload": cfg["name"], "form": "mixed" if mixed else "f64",
                              "setup_s": setup, "hierarchy_workspace_gb": h.ws.numel() / 1e9}), flush=True)
            forms = [("mixed", False), ("mixed+graphs", True)] if mixed else [("f64", False)]
            for name, graphs in forms:
                if mixed:
                    sd = m.solve_desc(tol=1e-10, kind="mg_mixed", smooth=args.smooth, smooth_coarse=args.smooth_coarse,
                                      coarse_iters=args.coarse_iters, inner_tol=args.inner_tol, maxiter=5000,
                                      coarse_bf16=True, smoother_f16=True, graphs=graphs)
                else:
                    sd = m.solve_desc(tol=1e-10, kind="mg", smooth=6, smooth_coarse=2, coarse_iters=1, maxiter=5000)
                ctx.autotune(bool(mixed))
                for n in sizes:
                    s_, d_, _ = h.level_info(0)
                    b = m.draw_z4(ctx, cfg["pseed"] + 950, 0, 0, n, s_, d_, "f64")
                    h.solve(0, b, sd)
                    torch.cuda.synchronize()
                    t0 = time.time()
                    x, st = h.solve(0, b, sd)
                    torch.cuda.synchronize()
                    dt = time.time() - t0
                    r = b - op.apply(x, prec="f64")
                    rel_res = (r.abs().pow(2).sum(dim=(0, 1)) / b.abs().pow(2).sum(dim=(0, 1))).sqrt()
                    ok = int((rel_res <= 1e-10).sum().item())
                    print(json.dumps({"study": "solve", "form": name, "nrhs": n, "seconds": dt,
                                      "rhs_per_s": ok / dt, "rhs_counted": ok, "iterations": st["iterations"],
                                      "iterations_per_rhs": st["iterations"] / n,
                                      "max_true_rel_residual": rel_res.max().item()}), flush=True)
                    del b, x, r
                ctx.autotune(False)
            del h
            torch.cuda.empty_cache()


def per_level_rates(m, ctx, h, cfg, sd, batch, torch):
    """RHS solved per second on each level alone: one batch of the level's
    size of Z4 right-hand sides solved to 1e-10 with the timed form's
    settings (after one untimed solve of the same batch)."""
    out = []
    for l in range(h.L):
        s_, d_, n_ = h.level_info(l)
        b = m.draw_z4(ctx, cfg["pseed"] + 900 + l, 256 * l, 0, batch[l], s_, d_, "f64")
        h.solve(l, b, sd)
        torch.cuda.synchronize()
        t0 = time.time()
        x, st = h.solve(l, b, sd)
        torch.cuda.synchronize()
        dt = time.time() - t0
        out.append({"level": l, "lattice_sites": s_, "dof": d_, "nrhs": batch[l], "seconds": dt,
                    "rhs_per_s": batch[l] / dt, "iterations": st["iterations"],
                    "max_rel_residual": st["max_rel_residual"]})
        del b, x
    return out


def micro(args):
    """Times one kernel alone: the fine dslash at the workload's lattice for
    one precision and rhs count (HIP events on the library's stream), or a
    plain 1 GiB device copy whose HBM counters calibrate the profiler's
    FETCH_SIZE / WRITE_SIZE readings."""
    import torch
    if args.micro == "copy":
        n = 1 << 27  # 2^27 doubles = 1 GiB
        x = torch.ones(n, dtype=torch.float64, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.iters):
            y.copy_(x)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.iters
        print(json.dumps({"micro": "copy", "bytes_read": 8 * n, "bytes_written": 8 * n, "avg_ms": ms,
                          "GBps": 16 * n / ms / 1e6}), flush=True)
        return
    cfg = CONFIGS[args.config]
    from lattice_inputs import gauge_field
    import paper_2509_11424_amd as m
    U = gauge_field(cfg["dims"], cfg["eps"], cfg["gseed"])
    ctx = m.Context(0)
    op = m.Operator(ctx, U, cfg["m0"], cfg["csw"])
    g = torch.Generator(device="cuda:0").manual_seed(5)
    if args.micro == "coarse":
        micro_coarse(args, cfg, m, ctx, op, g, torch)
        return
    for prec in args.prec.split(","):
        for nrhs in [int(v) for v in args.nrhs.split(",")]:
            shape = (12, op.V, nrhs)
            if prec == "f16":
                x = torch.randn(shape + (2,), generator=g, device="cuda:0").to(torch.float16)
            else:
                x = torch.randn(shape, generator=g, device="cuda:0",
                                dtype=torch.complex128 if prec == "f64" else torch.complex64)
            y = torch.empty_like(x)
            if args.micro == "step":
                xv = torch.zeros_like(x)
                wqr = torch.full((nrhs,), 0.01, dtype=torch.complex128, device="cuda:0")
                wqq = torch.ones(nrhs, dtype=torch.float64, device="cuda:0")

            def once():
                if args.micro == "dslash_dot":
                    op.apply_dot(x, y, prec)
                elif args.micro == "step":
                    op.smoother_step(x, xv, wqr, wqq, r_next=y)
                else:
                    op.apply(x, y, prec)

            key = "%s/%d/%d/%d" % ({"dslash_dot": "dslash_dot", "step": "dslash_step"}.get(args.micro, "dslash"),
                                   m.api.PREC[prec], op.V, nrhs)
            if args.variant is not None:
                ctx.tune_set(key, args.variant)
            if args.tune:
                ctx.autotune(True)
            for _ in range(3):
                once()
            ctx.autotune(False)
            torch.cuda.synchronize()
            ctx.profile(True)
            ctx.profile_reset()
            for _ in range(args.iters):
                once()
            torch.cuda.synchronize()
            q = ctx.profile_query("dslash_step" if args.micro == "step" else "dslash_" + prec)
            ctx.profile(False)
            ms = q["ms"] / q["launches"]
            bl = q["bytes"] / q["launches"]
            line = {"micro": args.micro, "prec": prec, "nrhs": nrhs, "lattice": "x".join(
                map(str, cfg["dims"])), "launches": q["launches"], "avg_ms": ms, "bytes_per_launch": bl,
                "GBps": bl / ms / 1e6, "frac": bl / ms / 1e6 / HBM_PEAK_GBS}
            rep = ctx.tune_report().get(key)
            if rep is not None:
                line["variant"], line["variant_ms"] = rep[0], rep[1]
            print(json.dumps(line), flush=True)
            del x, y


LEARNED = dict(widths=(4, 16, 16, 16, 4), train_seeds=list(range(1001, 1009)), eval_seeds=list(range(2001, 2009)),
               eps=0.6, m0=0.01, csw=1.0, dims=(16, 16, 16, 16), blocks=[(2, 2, 2, 2)], ntv=[12],
               big_dims=(24, 24, 24, 48), big_blocks=[(4, 4, 4, 4), (2, 2, 2, 2)], big_ntv=[24, 32],
               big_eval_seeds=list(range(2001, 2003)), pairs=16, epochs=4, steps_per_visit=15, lr=3e-3)


def learned_form(m, ctx, args, torch):
    """The learned-preconditioner form on its own workloads: a PTC network of
    four layers, 4 -> 16 -> 16 -> 16 -> 4 colour-triplet channels (one spinor's
    12 complex components in and out), BF16 weights with FP32 accumulation,
    trained with the library's kernels (full-batch Adam) on residual / error
    pairs from FP64 MG solves on 8 seeded 16^4 training fields (roughness 0.6,
    m0 0.01, c_sw 1; seeds 1001-1008), visiting the fields in turn for a few
    Adam steps each.  Then used as the fine smoother inside the mixed FGMRES
    on 8 held-out 16^4 fields (seeds 2001-2008) and on 24^3 x 48 fields, the
    weights carried over unchanged (the layers do not depend on the volume),
    against MR smoothing in the same solver and against plain FP64 MG, every
    solve to a true FP64 residual of 1e-10.  Returns the weights as a list."""
    import numpy as np
    from lattice_inputs import gauge_field
    L5 = LEARNED
    out = {"widths": list(L5["widths"]), "bf16_weights": True, "train_lattice": "x".join(map(str, L5["dims"])),
           "train_fields": L5["train_seeds"], "pairs_per_field": L5["pairs"], "epochs": L5["epochs"],
           "adam_steps_per_visit": L5["steps_per_visit"]}
    hs = []
    for sd_ in L5["train_seeds"]:
        U = gauge_field(L5["dims"], L5["eps"], sd_)
        op = m.Operator(ctx, U, L5["m0"], L5["csw"])
        h = m.Hierarchy(op, L5["blocks"], L5["ntv"], seed=sd_ + 100, max_nrhs=L5["pairs"], restart=16, mixed=2)
        hs.append((op, h))
    net0 = m.Net(hs[0][0], widths=L5["widths"], seed=3001, max_nrhs=L5["pairs"], train_nrhs=L5["pairs"],
                 bf16_weights=True)
    torch.cuda.synchronize()
    t0 = time.time()
    hist = []
    for ep in range(L5["epochs"]):
        for i, (op, h) in enumerate(hs):
            # the weights are field independent: each visit moves the network
            # to the field's links and trains on that field's pairs (Adam
            # state kept across visits)
            net0.bind(op)
            tr = net0.train(h, steps=L5["steps_per_visit"], lr=L5["lr"], seed=4000 + 100 * ep + i,
                            target_tol=1e-8)
            hist.append([tr["loss_first"], tr["loss_last"]])
    torch.cuda.synchronize()
    out["train_s"] = time.time() - t0
    out["loss_first"] = hist[0][0]
    out["loss_last"] = hist[-1][1]
    weights = net0.get_weights()
    del net0, hs
    torch.cuda.empty_cache()

    def settings(kind, net=None):
        if kind == "f64":
            return m.solve_desc(tol=1e-10, kind="mg", smooth=6, smooth_coarse=2, coarse_iters=1, maxiter=5000)
        return m.solve_desc(tol=1e-10, kind=kind, net=net, smooth=args.smooth, smooth_coarse=args.smooth_coarse,
                            coarse_iters=args.coarse_iters, inner_tol=args.inner_tol, maxiter=5000,
                            coarse_bf16=True, smoother_f16=True, graphs=True)

    def evaluate(dims, blocks, ntv, seeds, nrhs):
        rows = []
        for sd_ in seeds:
            U = gauge_field(dims, L5["eps"], sd_)
            op = m.Operator(ctx, U, L5["m0"], L5["csw"])
            h = m.Hierarchy(op, blocks, ntv, seed=sd_ + 100, max_nrhs=nrhs, restart=12, mixed=2)
            net = m.Net(op, widths=L5["widths"], seed=1, max_nrhs=nrhs, bf16_weights=True)
            net.set_weights(weights)
            s_, d_, _ = h.level_info(0)
            b = m.draw_z4(ctx, sd_ + 5000, 0, 0, nrhs, s_, d_, "f64")
            row = {"seed": sd_}
            for name, sd in (("mr", settings("mg_mixed")), ("net", settings("net", net)), ("f64", settings("f64"))):
                h.solve(0, b, sd)  # warm-up: autotuning, graph capture
                torch.cuda.synchronize()
                t1 = time.time()
                x, st = h.solve(0, b, sd)
                torch.cuda.synchronize()
                row[name] = {"seconds": time.time() - t1, "iterations": st["iterations"],
                             "fallbacks": st["fallbacks"], "max_rel_residual": st["max_rel_residual"]}
            # traces: the same probes through both smoothers
            npr = [4] * h.L
            a = h.estimate("trace", "orthogonal", npr, seed=sd_ + 6000, batch=nrhs, solve=settings("net", net))
            c = h.estimate("trace", "orthogonal", npr, seed=sd_ + 6000, batch=nrhs, solve=settings("mg_mixed"))
            d = max(float(np.max(np.abs(sa - sc)) / max(np.max(np.abs(sc)), 1e-300))
                    for sa, sc in zip(a["samples"], c["samples"]))
            row["trace_max_rel_diff"] = d
            row["trace_net"] = [a["total_mean"][0, 0].real, a["total_mean"][0, 0].imag]
            rows.append(row)
            del h, net, op, b
            torch.cuda.empty_cache()
        return rows

    out["eval_16x16x16x16"] = evaluate(L5["dims"], L5["blocks"], L5["ntv"], L5["eval_seeds"], L5["pairs"])
    out["eval_24x24x24x48"] = evaluate(L5["big_dims"], L5["big_blocks"], L5["big_ntv"], L5["big_eval_seeds"],
                                       L5["pairs"])
    for key in ("eval_16x16x16x16", "eval_24x24x24x48"):
        rows = out[key]
        out[key + "_mean"] = {n: {"seconds": float(np.mean([r[n]["seconds"] for r in rows])),
                                  "iterations": float(np.mean([r[n]["iterations"] for r in rows]))}
                              for n in ("mr", "net", "f64")}
    return out, weights


def time_to_target(m, ctx, op, cfg, make_mixed, sd_mixed, args, weights=None):
    """Time to reach the variance of the plain FP64 orthogonal estimate at the
    configured probe counts (target eps^2), for plain FP64 MG and for the
    mixed form with MLMC-optimal sample sizes (Sec. 2.2, eq. MLMC-Nl); with
    trained network weights also for the learned form (the mixed form with
    the network as the fine smoother)."""
    import numpy as np
    import torch
    L = len(cfg["nprobe"])
    lv = list(range(L - 1)) + list(range(L - 1)) + [L - 1]

    def pilot(h, sd, batch):
        torch.cuda.synchronize()
        t0 = time.time()
        r = h.estimate("trace", "orthogonal", cfg["nprobe"], seed=cfg["pseed"] + 7, batch=batch,
                       solve=sd, samples=False)
        torch.cuda.synchronize()
        return {"seconds": time.time() - t0, "var": r["var"][:, 0, 0], "cost": r["cost_s"],
                "total_var": float(r["total_var"][0, 0])}

    def final(h, sd, p, eps2, batch):
        # MLMC-optimal N per term; terms of one probe group share the largest
        n = m.mlmc_allocate(np.maximum(p["var"], 1e-30), np.maximum(p["cost"], 1e-9), eps2)
        npl = [int(max(n[i] for i in range(len(lv)) if lv[i] == g)) for g in range(L)]
        torch.cuda.synchronize()
        t0 = time.time()
        r = h.estimate("trace", "orthogonal", npl, seed=cfg["pseed"] + 11, batch=batch, solve=sd,
                       samples=False)
        torch.cuda.synchronize()
        return {"seconds": time.time() - t0, "nprobe": npl, "achieved_var": float(r["total_var"][0, 0]),
                "pilot_seconds": p["seconds"]}

    # one hierarchy at a time: the FP64 one first (its pilot fixes eps^2, the
    # variance of the plain FP64 estimate at the configured probe counts),
    # then the mixed one, built anew
    b64 = cfg.get("batch_f64", cfg["batch"])
    h64 = m.Hierarchy(op, cfg["blocks"], cfg["ntv"], seed=cfg["pseed"] + 1000, max_nrhs=b64[0],
                      max_nrhs_level=b64, restart=cfg["restart"], mixed=0)
    sd64 = m.solve_desc(tol=1e-10, kind="mg", smooth=6, smooth_coarse=2, coarse_iters=1, maxiter=5000)
    p64 = pilot(h64, sd64, b64)
    progress("time to target: FP64 pilot %.1f s" % p64["seconds"])
    eps2 = p64["total_var"]
    out = {"eps2": eps2, "f64": final(h64, sd64, p64, eps2, b64)}
    out["f64"]["batch"] = b64
    del h64
    torch.cuda.empty_cache()
    h_mixed = make_mixed()
    pm = pilot(h_mixed, sd_mixed, cfg["batch"])
    progress("time to target: mixed pilot %.1f s" % pm["seconds"])
    out["mixed"] = final(h_mixed, sd_mixed, pm, eps2, cfg["batch"])
    out["mixed"]["batch"] = cfg["batch"]
    if weights is not None:
        net = m.Net(op, widths=LEARNED["widths"], seed=1, max_nrhs=cfg["batch"][0], bf16_weights=True)
        net.set_weights(weights)
        sd_net = m.solve_desc(tol=1e-10, kind="net", net=net, smooth=sd_mixed.smooth,
                              smooth_coarse=sd_mixed.smooth_coarse, coarse_iters=sd_mixed.coarse_iters,
                              inner_tol=sd_mixed.inner_tol, maxiter=5000, coarse_bf16=True, smoother_f16=True,
                              graphs=True)
        pn = pilot(h_mixed, sd_net, cfg["batch"])
        out["learned"] = final(h_mixed, sd_net, pn, eps2, cfg["batch"])
        out["learned"]["batch"] = cfg["batch"]
        out["ratio_f64_over_learned"] = out["f64"]["seconds"] / out["learned"]["seconds"]
        del net
    del h_mixed
    torch.cuda.empty_cache()
    out["ratio_f64_over_mixed"] = out["f64"]["seconds"] / out["mixed"]["seconds"]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c4", choices=sorted(CONFIGS))
    ap.add_argument("--smooth", type=int, default=9, help="fine-level smoothing steps of the timed form")
    ap.add_argument("--smooth-coarse", type=int, default=3, help="smoothing steps on the coarser levels")
    ap.add_argument("--coarse-iters", type=int, default=1, help="FGMRES steps of a coarse-grid solve")
    ap.add_argument("--inner-tol", type=float, default=6e-3,
                    help="residual reduction of each FP32 inner solve of the mixed form")
    ap.add_argument("--batch", type=int, nargs="+", default=None,
                    help="right-hand sides per batch on each level (default: the configuration's)")
    ap.add_argument("--form", default="mixed", choices=["mixed", "f64"])
    ap.add_argument("--cpu", type=int, default=1)
    ap.add_argument("--ttt", type=int, default=1, help="time to target variance, FP64 against the mixed form")
    ap.add_argument("--learned", action="store_true", help="also measure the learned-preconditioner form")
    ap.add_argument("--cpu-study", action="store_true",
                    help="the FP64 oracle on the host cores at the small workloads (no GPU)")
    ap.add_argument("--hierarchy-study", action="store_true",
                    help="per-term variance against setup cost for N_tv 64 and refined test vectors")
    ap.add_argument("--observables", action="store_true",
                    help="estimate C(t) three ways and the loops two ways with the timed form, one line each")
    ap.add_argument("--obs-probes", type=int, nargs="+", default=None,
                    help="observables: probes per group (default: the configuration's)")
    ap.add_argument("--solve-study", action="store_true",
                    help="RHS/s to 1e-10 on the fine level over batch size (--nrhs, default 12,32,64) and form")
    ap.add_argument("--micro", choices=["dslash", "dslash_dot", "step", "copy", "coarse"])
    ap.add_argument("--level", type=int, default=1, help="micro coarse: hierarchy level of the stencil")
    ap.add_argument("--tune", action="store_true", help="micro: autotune the launch shape first")
    ap.add_argument("--variant", type=int, default=None, help="micro: pin this launch variant")
    ap.add_argument("--prec", default="f32", help="comma list of f64, f32, f16")
    ap.add_argument("--nrhs", default=None, help="comma list of rhs counts (micro: default 8)")
    ap.add_argument("--iters", type=int, default=50)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the hot path is measured on one GPU's share of the "
              "probes (probes shard across GPUs without communication until the final sums); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.micro:
        args.nrhs = args.nrhs or "8"
        micro(args)
    elif args.observables:
        observables(args)
    elif args.hierarchy_study:
        hierarchy_study(args)
    elif args.cpu_study:
        cpu_study(args)
    elif args.solve_study:
        solve_study(args)
    else:
        run(args)


if __name__ == "__main__":
    main()
