"""Python binding of the mgmlmc C ABI (include/mgmlmc.h).

Argument marshalling only: every computation runs in the HIP library.  torch
provides the device memory (workspaces, vectors) and the HIP stream.  Vectors
are complex torch tensors in the library's dof-major layout, shape
(dof, sites, nrhs); `to_dofmajor` / `from_dofmajor` convert from the natural
(nrhs, sites, dof) layout.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmgmlmc.so")

MAX_LEVELS = 4
PREC = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3}
SOLVE = {"mg": 0, "mg_mixed": 1, "gmres": 2, "net": 3}
OBS = {"trace": 0, "corr": 1, "loops": 2}
DEC = {"plain": 0, "oblique": 1, "orthogonal": 2, "deflated": 3}
EXPORT = {"agg_map": 0, "P": 1, "coarse": 2, "tv": 3}
NOISE = {"z4": 0, "z2": 1, "u1": 2, "gauss": 3}
KCLASS = {"dslash_f64": 0, "dslash_f32": 1, "dslash_f16": 2, "coarse_f64": 3, "coarse_f32": 4,
          "coarse_bf16": 5, "transfer": 6, "net": 7, "dslash_step": 8}
NET_MAX_LAYERS = 8
NOALLOC_SCRATCH_BYTES = 16 << 20  # MGM_NOALLOC_SCRATCH_BYTES
STATUS = {0: "MGM_OK", -1: "MGM_ERR_INVALID_ARG", -2: "MGM_ERR_SHAPE", -3: "MGM_ERR_WORKSPACE",
          -4: "MGM_ERR_NOT_CONVERGED", -5: "MGM_ERR_RANK_DEFICIENT", -6: "MGM_ERR_NUMERIC",
          -7: "MGM_ERR_HIP"}


class MgmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class LatticeDesc(C.Structure):
    _fields_ = [("dims", C.c_int32 * 4), ("m0", C.c_double), ("csw", C.c_double),
                ("t_antiperiodic", C.c_int32)]


class HierarchyDesc(C.Structure):
    _fields_ = [("nlevels", C.c_int32), ("block", (C.c_int32 * 4) * (MAX_LEVELS - 1)),
                ("ntv", C.c_int32 * (MAX_LEVELS - 1)), ("setup_steps", C.c_int32),
                ("setup_mr", C.c_int32), ("seed", C.c_uint64), ("max_nrhs", C.c_int32),
                ("restart", C.c_int32), ("mixed", C.c_int32), ("with_corr", C.c_int32),
                ("max_nrhs_level", C.c_int32 * MAX_LEVELS)]


class SolveDesc(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxiter", C.c_int32), ("kind", C.c_int32),
                ("smooth", C.c_int32), ("coarse_iters", C.c_int32), ("inner_tol", C.c_double),
                ("net", C.c_void_p), ("coarse_bf16", C.c_int32), ("smoother_f16", C.c_int32),
                ("smooth_coarse", C.c_int32), ("graphs", C.c_int32)]


class RefineDesc(C.Structure):
    _fields_ = [("max_iters", C.c_int32), ("eig_tol", C.c_double), ("power_tol", C.c_double),
                ("batch", C.c_int32), ("solve", SolveDesc)]


class RefineStats(C.Structure):
    _fields_ = [("steps", C.c_int32), ("converged", C.c_int32), ("max_rho_start", C.c_double),
                ("max_rho", C.c_double), ("seconds", C.c_double)]


class SolveStats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("restarts", C.c_int32), ("fallbacks", C.c_int32),
                ("max_rel_residual", C.c_double), ("seconds", C.c_double)]


class EstimateDesc(C.Structure):
    _fields_ = [("observable", C.c_int32), ("decomposition", C.c_int32),
                ("nprobe", C.c_int32 * MAX_LEVELS), ("seed", C.c_uint64),
                ("first_probe", C.c_uint64), ("batch", C.c_int32), ("solve", SolveDesc),
                ("batch_level", C.c_int32 * MAX_LEVELS), ("deflation", C.c_void_p), ("noise", C.c_int32),
                ("probing", C.c_int32)]


class DeflationDesc(C.Structure):
    _fields_ = [("k", C.c_int32), ("power_iters", C.c_int32), ("power_tol", C.c_double), ("seed", C.c_uint64),
                ("batch", C.c_int32), ("solve", SolveDesc)]


class EstimateSizes(C.Structure):
    _fields_ = [("nterms", C.c_int32), ("T", C.c_int32), ("ngamma", C.c_int32),
                ("nsamples", C.c_int64)]


class EstimateResult(C.Structure):
    _fields_ = [("n", C.POINTER(C.c_int64)), ("mean", C.POINTER(C.c_double)),
                ("var", C.POINTER(C.c_double)), ("cost_s", C.POINTER(C.c_double)),
                ("samples", C.POINTER(C.c_double)), ("total_mean", C.POINTER(C.c_double)),
                ("total_var", C.POINTER(C.c_double)), ("stats", SolveStats)]


class NetDesc(C.Structure):
    _fields_ = [("nlayers", C.c_int32), ("width", C.c_int32 * (NET_MAX_LAYERS + 1)), ("seed", C.c_uint64),
                ("max_nrhs", C.c_int32), ("train_nrhs", C.c_int32), ("bf16_weights", C.c_int32)]


class TrainDesc(C.Structure):
    _fields_ = [("steps", C.c_int32), ("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double),
                ("eps", C.c_double), ("seed", C.c_uint64), ("target_tol", C.c_double)]


class TrainStats(C.Structure):
    _fields_ = [("loss_first", C.c_double), ("loss_last", C.c_double), ("steps", C.c_int32),
                ("seconds", C.c_double)]


_lib = None

# (name, restype, argtypes)
_SIGS = [
    ("mgm_status_string", C.c_char_p, [C.c_int]),
    ("mgm_last_error", C.c_char_p, []),
    ("mgm_version", C.c_char_p, []),
    ("mgm_context_create", C.c_int, [C.c_int, C.c_void_p, C.POINTER(C.c_void_p)]),
    ("mgm_context_set_stream", C.c_int, [C.c_void_p, C.c_void_p]),
    ("mgm_context_set_autotune", C.c_int, [C.c_void_p, C.c_int32]),
    ("mgm_context_tune_report", C.c_int, [C.c_void_p, C.c_char_p, C.c_size_t, C.POINTER(C.c_size_t)]),
    ("mgm_context_tune_set", C.c_int, [C.c_void_p, C.c_char_p, C.c_int32]),
    ("mgm_context_destroy", None, [C.c_void_p]),
    ("mgm_operator_workspace_size", C.c_int, [C.POINTER(LatticeDesc), C.POINTER(C.c_size_t)]),
    ("mgm_operator_create", C.c_int, [C.c_void_p, C.POINTER(LatticeDesc), C.c_void_p, C.c_void_p,
                                      C.c_size_t, C.POINTER(C.c_void_p)]),
    ("mgm_operator_apply", C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int32]),
    ("mgm_operator_sites", C.c_int64, [C.c_void_p]),
    ("mgm_operator_destroy", None, [C.c_void_p]),
    ("mgm_draw_z4", C.c_int, [C.c_void_p, C.c_uint64, C.c_uint32, C.c_uint64, C.c_int32, C.c_int64,
                              C.c_int32, C.c_int, C.c_void_p]),
    ("mgm_draw_noise", C.c_int, [C.c_void_p, C.c_int32, C.c_uint64, C.c_uint32, C.c_uint64, C.c_int32, C.c_int64,
                                 C.c_int32, C.c_int, C.c_void_p]),
    ("mgm_hierarchy_workspace_size", C.c_int, [C.c_void_p, C.POINTER(HierarchyDesc),
                                               C.POINTER(C.c_size_t)]),
    ("mgm_hierarchy_create", C.c_int, [C.c_void_p, C.POINTER(HierarchyDesc), C.c_void_p, C.c_size_t,
                                       C.POINTER(C.c_void_p)]),
    ("mgm_hierarchy_level_info", C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int64),
                                           C.POINTER(C.c_int32), C.POINTER(C.c_int64)]),
    ("mgm_hierarchy_export", C.c_int, [C.c_void_p, C.c_int32, C.c_int, C.c_void_p, C.c_size_t]),
    ("mgm_level_apply", C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32]),
    ("mgm_level_apply_prec", C.c_int, [C.c_void_p, C.c_int32, C.c_int, C.c_void_p, C.c_void_p,
                                       C.c_int32]),
    ("mgm_restrict", C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32]),
    ("mgm_prolong", C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32]),
    ("mgm_project_out", C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32]),
    ("mgm_restrict_prec", C.c_int, [C.c_void_p, C.c_int32, C.c_int, C.c_void_p, C.c_void_p, C.c_int32]),
    ("mgm_prolong_prec", C.c_int, [C.c_void_p, C.c_int32, C.c_int, C.c_void_p, C.c_void_p, C.c_int32]),
    ("mgm_restrict_f16", C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]),
    ("mgm_prolong_add_f16", C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_int32]),
    ("mgm_solve", C.c_int, [C.c_void_p, C.c_int32, C.POINTER(SolveDesc), C.c_void_p, C.c_void_p,
                            C.c_int32, C.POINTER(SolveStats)]),
    ("mgm_estimate_sizes_query", C.c_int, [C.c_void_p, C.POINTER(EstimateDesc),
                                           C.POINTER(EstimateSizes)]),
    ("mgm_estimate", C.c_int, [C.c_void_p, C.POINTER(EstimateDesc), C.POINTER(EstimateResult)]),
    ("mgm_mlmc_allocate", C.c_int, [C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                    C.c_double, C.POINTER(C.c_int64)]),
    ("mgm_profile_enable", C.c_int, [C.c_void_p, C.c_int32]),
    ("mgm_profile_reset", C.c_int, [C.c_void_p]),
    ("mgm_profile_query", C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int64),
                                    C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    ("mgm_hierarchy_destroy", None, [C.c_void_p]),
    ("mgm_operator_dot_workspace_size", C.c_int, [C.c_void_p, C.c_int, C.c_int32, C.POINTER(C.c_size_t)]),
    ("mgm_operator_apply_dot", C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                                         C.c_size_t, C.c_void_p, C.c_void_p]),
    ("mgm_operator_apply_dot_noalloc", C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int32,
                                                 C.c_void_p, C.c_void_p]),
    ("mgm_operator_smoother_step", C.c_int, [C.c_void_p] * 6 + [C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p,
                                                                C.c_void_p]),
    ("mgm_operator_step_fusable", C.c_int32, [C.c_void_p, C.c_int32]),
    ("mgm_hierarchy_refine_workspace_size", C.c_int, [C.c_void_p, C.POINTER(C.c_size_t)]),
    ("mgm_hierarchy_refine", C.c_int, [C.c_void_p, C.POINTER(RefineDesc), C.c_void_p, C.c_size_t,
                                       C.POINTER(RefineStats), C.c_void_p, C.c_void_p]),
    ("mgm_deflation_workspace_size", C.c_int, [C.c_void_p, C.POINTER(DeflationDesc), C.POINTER(C.c_size_t)]),
    ("mgm_deflation_create", C.c_int, [C.c_void_p, C.POINTER(DeflationDesc), C.c_void_p, C.c_size_t,
                                       C.POINTER(C.c_void_p)]),
    ("mgm_deflation_export", C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    ("mgm_deflation_info", C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                     C.POINTER(C.c_double)]),
    ("mgm_deflation_destroy", None, [C.c_void_p]),
    ("mgm_net_workspace_size", C.c_int, [C.c_void_p, C.POINTER(NetDesc), C.POINTER(C.c_size_t)]),
    ("mgm_net_create", C.c_int, [C.c_void_p, C.POINTER(NetDesc), C.c_void_p, C.c_size_t,
                                 C.POINTER(C.c_void_p)]),
    ("mgm_net_bind", C.c_int, [C.c_void_p, C.c_void_p]),
    ("mgm_net_num_weights", C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    ("mgm_net_save", C.c_int, [C.c_void_p, C.c_char_p]),
    ("mgm_net_load", C.c_int, [C.c_void_p, C.c_char_p]),
    ("mgm_net_set_weights", C.c_int, [C.c_void_p, C.c_void_p]),
    ("mgm_net_get_weights", C.c_int, [C.c_void_p, C.c_void_p]),
    ("mgm_net_apply", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]),
    ("mgm_net_loss_grad", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(C.c_double),
                                    C.c_void_p]),
    ("mgm_net_train", C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(TrainDesc), C.POINTER(TrainStats),
                                C.c_void_p]),
    ("mgm_net_destroy", None, [C.c_void_p]),
]

EXPORTED = [s[0] for s in _SIGS]


def lib():
    """Loads the HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libmgmlmc.so is not built (run __graft_entry__.build() or "
                               "python -m paper_2509_11424_amd.build); there is no fallback")
        l = C.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            f = getattr(l, name)
            f.restype = res
            f.argtypes = args
        _lib = l
    return _lib


def _check(st: int):
    if st != 0:
        raise MgmError(st, lib().mgm_last_error().decode())


def _ptr(t) -> int:
    return t.data_ptr()


# ------------------------------------------------------------------ layout

def to_dofmajor(x: np.ndarray) -> np.ndarray:
    """(nrhs, sites, dof) -> (dof, sites, nrhs) contiguous."""
    return np.ascontiguousarray(np.transpose(x, (2, 1, 0)))


def from_dofmajor(x: np.ndarray) -> np.ndarray:
    """(dof, sites, nrhs) -> (nrhs, sites, dof) contiguous."""
    return np.ascontiguousarray(np.transpose(x, (2, 1, 0)))


def gauge_to_host(U: np.ndarray) -> np.ndarray:
    """(T, Z, Y, X, 4, 3, 3) complex128 -> contiguous float64 view for the ABI."""
    U = np.ascontiguousarray(U, dtype=np.complex128)
    return U.view(np.float64)


# ------------------------------------------------------------------ objects

class Context:
    def __init__(self, device: int = 0, stream=None):
        import torch
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device).cuda_stream
        h = C.c_void_p()
        _check(lib().mgm_context_create(device, C.c_void_p(stream), C.byref(h)))
        self.h = h

    def set_stream(self, stream):
        _check(lib().mgm_context_set_stream(self.h, C.c_void_p(stream)))

    def autotune(self, on: bool = True):
        _check(lib().mgm_context_set_autotune(self.h, 1 if on else 0))

    def tune_report(self) -> dict:
        """{key: (variant, [ms per variant])} of the tuned launch shapes."""
        need = C.c_size_t()
        _check(lib().mgm_context_tune_report(self.h, None, 0, C.byref(need)))
        buf = C.create_string_buffer(need.value)
        _check(lib().mgm_context_tune_report(self.h, buf, need.value, C.byref(need)))
        out = {}
        for line in buf.value.decode().splitlines():
            f = line.split()
            out[f[0]] = (int(f[1]), [float(v) for v in f[2:]])
        return out

    def tune_set(self, key: str, variant: int):
        """Pins launch variant `variant` for the tuned shape `key`."""
        _check(lib().mgm_context_tune_set(self.h, key.encode(), int(variant)))

    def profile(self, on: bool = True):
        _check(lib().mgm_profile_enable(self.h, 1 if on else 0))

    def profile_reset(self):
        _check(lib().mgm_profile_reset(self.h))

    def profile_query(self, kclass: str):
        n = C.c_int64()
        ms = C.c_double()
        by = C.c_double()
        _check(lib().mgm_profile_query(self.h, KCLASS[kclass], C.byref(n), C.byref(ms), C.byref(by)))
        return {"launches": n.value, "ms": ms.value, "bytes": by.value}

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.mgm_context_destroy(self.h)
            self.h = None


def _empty_ws(nbytes: int, device: int):
    import torch
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device="cuda:%d" % device)


class Operator:
    """Wilson-clover operator on the GPU built from an FP64 host gauge field."""

    def __init__(self, ctx: Context, gauge: np.ndarray, m0: float, csw: float,
                 antiperiodic_t: bool = True):
        T, Z, Y, X = gauge.shape[:4]
        self.ctx = ctx
        self.dims = (X, Y, Z, T)
        self.V = X * Y * Z * T
        d = LatticeDesc()
        d.dims[:] = [X, Y, Z, T]
        d.m0 = m0
        d.csw = csw
        d.t_antiperiodic = 1 if antiperiodic_t else 0
        self.desc = d
        nb = C.c_size_t()
        _check(lib().mgm_operator_workspace_size(C.byref(d), C.byref(nb)))
        self.ws = _empty_ws(nb.value, ctx.device)
        g = gauge_to_host(gauge)
        h = C.c_void_p()
        _check(lib().mgm_operator_create(ctx.h, C.byref(d), g.ctypes.data_as(C.c_void_p),
                                         C.c_void_p(_ptr(self.ws)), self.ws.numel(), C.byref(h)))
        self.h = h

    def apply(self, x, y=None, prec: str = "f64"):
        """y = D x; x is a dof-major tensor (12, V, nrhs) of the precision's dtype
        (f64: complex128, f32: complex64, f16: float16 pairs (12, V, nrhs, 2))."""
        import torch
        if y is None:
            y = torch.empty_like(x)
        nrhs = x.shape[2]
        _check(lib().mgm_operator_apply(self.h, PREC[prec], C.c_void_p(_ptr(x)), C.c_void_p(_ptr(y)),
                                        nrhs))
        return y

    def apply_dot(self, x, y=None, prec: str = "f64"):
        """y = D x with the fused per-rhs reductions; returns (y, y^H x, |y|^2)
        as (tensor, complex128 tensor (nrhs,), float64 tensor (nrhs,))."""
        import torch
        if y is None:
            y = torch.empty_like(x)
        nrhs = x.shape[2]
        nb = C.c_size_t()
        _check(lib().mgm_operator_dot_workspace_size(self.h, PREC[prec], nrhs, C.byref(nb)))
        ws = _empty_ws(nb.value, self.ctx.device)
        yx = torch.empty(nrhs, dtype=torch.complex128, device=x.device)
        yy = torch.empty(nrhs, dtype=torch.float64, device=x.device)
        _check(lib().mgm_operator_apply_dot(self.h, PREC[prec], C.c_void_p(_ptr(x)), C.c_void_p(_ptr(y)), nrhs,
                                            C.c_void_p(_ptr(ws)), ws.numel(), C.c_void_p(_ptr(yx)),
                                            C.c_void_p(_ptr(yy))))
        return y, yx, yy

    def apply_dot_noalloc(self, x, y, yx, yy, prec: str = "f64"):
        """mgm_operator_apply_dot_noalloc into caller tensors y (like x),
        yx (complex128 (nrhs,)) and yy (float64 (nrhs,)); allocates nothing."""
        _check(lib().mgm_operator_apply_dot_noalloc(self.h, PREC[prec], C.c_void_p(_ptr(x)), C.c_void_p(_ptr(y)),
                                                    x.shape[2], C.c_void_p(_ptr(yx)), C.c_void_p(_ptr(yy))))
        return y, yx, yy

    def dot_workspace_size(self, nrhs: int, prec: str = "f64") -> int:
        nb = C.c_size_t()
        _check(lib().mgm_operator_dot_workspace_size(self.h, PREC[prec], nrhs, C.byref(nb)))
        return nb.value

    def step_fusable(self, nrhs: int) -> bool:
        return bool(lib().mgm_operator_step_fusable(self.h, nrhs))

    def smoother_step(self, r, x, qr_prev, qq_prev, r_next=None):
        """One fused FP16 smoother step (float16 pair tensors (12, V, nrhs, 2);
        qr_prev complex128 / qq_prev float64 (nrhs,)): returns (r_next, q^H r,
        |q|^2) and updates x in place."""
        import torch
        nrhs = r.shape[2]
        if r_next is None:
            r_next = torch.empty_like(r)
        nb = C.c_size_t()
        _check(lib().mgm_operator_dot_workspace_size(self.h, PREC["f16"], nrhs, C.byref(nb)))
        ws = _empty_ws(nb.value, self.ctx.device)
        yx = torch.empty(nrhs, dtype=torch.complex128, device=r.device)
        yy = torch.empty(nrhs, dtype=torch.float64, device=r.device)
        _check(lib().mgm_operator_smoother_step(self.h, *[C.c_void_p(_ptr(t)) for t in (r, r_next, x, qr_prev,
                                                                                         qq_prev)],
                                                nrhs, C.c_void_p(_ptr(ws)), ws.numel(), C.c_void_p(_ptr(yx)),
                                                C.c_void_p(_ptr(yy))))
        return r_next, yx, yy

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.mgm_operator_destroy(self.h)
            self.h = None


def draw_z4(ctx: Context, seed: int, stream: int, first_probe: int, nprobe: int, nsite: int, dof: int,
            prec: str = "f64"):
    import torch
    dt = torch.complex128 if prec == "f64" else torch.complex64
    out = torch.empty((dof, nsite, nprobe), dtype=dt, device="cuda:%d" % ctx.device)
    _check(lib().mgm_draw_z4(ctx.h, seed, stream, first_probe, nprobe, nsite, dof, PREC[prec],
                             C.c_void_p(_ptr(out))))
    return out


def draw_noise(ctx: Context, kind, seed: int, stream: int, first_probe: int, nprobe: int, nsite: int, dof: int,
               prec: str = "f64"):
    """Probe entries of distribution kind ("z4", "z2", "u1", "gauss")."""
    import torch
    dt = torch.complex128 if prec == "f64" else torch.complex64
    out = torch.empty((dof, nsite, nprobe), dtype=dt, device="cuda:%d" % ctx.device)
    k = NOISE[kind] if isinstance(kind, str) else int(kind)
    _check(lib().mgm_draw_noise(ctx.h, k, seed, stream, first_probe, nprobe, nsite, dof, PREC[prec],
                                C.c_void_p(_ptr(out))))
    return out


def solve_desc(tol=1e-12, maxiter=2000, kind="mg", smooth=2, coarse_iters=8, inner_tol=1e-5,
               net=None, coarse_bf16=True, smoother_f16=True, graphs=False, smooth_coarse=0) -> SolveDesc:
    d = SolveDesc()
    d.smooth_coarse = smooth_coarse
    d.graphs = 1 if graphs else 0
    d.coarse_bf16 = 1 if coarse_bf16 else 0
    d.smoother_f16 = 1 if smoother_f16 else 0
    d.tol = tol
    d.maxiter = maxiter
    d.kind = SOLVE[kind] if isinstance(kind, str) else int(kind)
    d.smooth = smooth
    d.coarse_iters = coarse_iters
    d.inner_tol = inner_tol
    d.net = net.h if net is not None else None
    return d


class Hierarchy:
    def __init__(self, op: Operator, blocks, ntv, seed: int, setup_steps: int = 20, setup_mr: int = 4,
                 max_nrhs: int = 8, restart: int = 16, mixed: int = 0, with_corr: bool = False,
                 max_nrhs_level=None):
        self.op = op
        self.ctx = op.ctx
        d = HierarchyDesc()
        d.nlevels = len(blocks) + 1
        for l, b in enumerate(blocks):
            d.block[l][:] = list(b)
            d.ntv[l] = ntv[l]
        d.setup_steps = setup_steps
        d.setup_mr = setup_mr
        d.seed = seed
        d.max_nrhs = max_nrhs
        d.restart = restart
        d.mixed = mixed
        d.with_corr = 1 if with_corr else 0
        if max_nrhs_level is not None:
            caps = list(max_nrhs_level) + [0] * (MAX_LEVELS - len(max_nrhs_level))
            d.max_nrhs_level[:] = caps[:MAX_LEVELS]
        self.desc = d
        self.L = d.nlevels
        nb = C.c_size_t()
        _check(lib().mgm_hierarchy_workspace_size(op.h, C.byref(d), C.byref(nb)))
        self.ws_bytes = nb.value
        self.ws = _empty_ws(nb.value, self.ctx.device)
        h = C.c_void_p()
        _check(lib().mgm_hierarchy_create(op.h, C.byref(d), C.c_void_p(_ptr(self.ws)), self.ws.numel(),
                                          C.byref(h)))
        self.h = h

    def refine(self, max_iters: int = 20, eig_tol: float = 1e-4, power_tol: float = 1e-6, batch: int | None = None,
               solve: SolveDesc | None = None) -> dict:
        """Replaces the fine test vectors by Ritz vectors of Gamma5 D refined
        to eigen-residual eig_tol and rebuilds the hierarchy in place."""
        d = RefineDesc()
        d.max_iters, d.eig_tol, d.power_tol = max_iters, eig_tol, power_tol
        cap = self.desc.max_nrhs_level[0] or self.desc.max_nrhs
        d.batch = batch if batch is not None else min(cap, self.desc.ntv[0])
        d.solve = solve or solve_desc()
        nb = C.c_size_t()
        _check(lib().mgm_hierarchy_refine_workspace_size(self.h, C.byref(nb)))
        ws = _empty_ws(nb.value, self.ctx.device)
        st = RefineStats()
        k = self.desc.ntv[0]
        rho = np.zeros(k)
        theta = np.zeros(k)
        _check(lib().mgm_hierarchy_refine(self.h, C.byref(d), C.c_void_p(_ptr(ws)), ws.numel(), C.byref(st),
                                          rho.ctypes.data_as(C.c_void_p), theta.ctypes.data_as(C.c_void_p)))
        del ws
        return {"steps": st.steps, "converged": bool(st.converged), "max_rho_start": st.max_rho_start,
                "max_rho": st.max_rho, "seconds": st.seconds, "rho": rho, "theta": theta}

    def level_info(self, level: int):
        s = C.c_int64()
        d = C.c_int32()
        n = C.c_int64()
        _check(lib().mgm_hierarchy_level_info(self.h, level, C.byref(s), C.byref(d), C.byref(n)))
        return s.value, d.value, n.value

    def export(self, level: int, what: str) -> np.ndarray:
        sites, dof, n = self.level_info(level)
        cs, cd, cn = self.level_info(level + 1)
        ntv = cd // 2
        rows = (sites // cs) * (dof // 2)
        if what == "agg_map":
            out = np.zeros((cs, 2, rows), dtype=np.int64)
        elif what == "P":
            out = np.zeros((cs, 2, rows, ntv), dtype=np.complex128)
        elif what == "coarse":
            out = np.zeros((cs, 9, cd, cd), dtype=np.complex128)
        elif what == "tv":
            out = np.zeros((ntv, n), dtype=np.complex128)
        else:
            raise ValueError(what)
        _check(lib().mgm_hierarchy_export(self.h, level, EXPORT[what], out.ctypes.data_as(C.c_void_p),
                                          out.nbytes))
        return out

    def _vec(self, level: int, nrhs: int, dtype=None):
        import torch
        s, d, _ = self.level_info(level)
        return torch.empty((d, s, nrhs), dtype=dtype or torch.complex128, device="cuda:%d" % self.ctx.device)

    def apply(self, level: int, x):
        y = self._vec(level, x.shape[2])
        _check(lib().mgm_level_apply(self.h, level, C.c_void_p(_ptr(x)), C.c_void_p(_ptr(y)), x.shape[2]))
        return y

    def apply_prec(self, level: int, x, prec: str):
        """Level operator in precision prec; x: complex64 (f32, bf16) or
        complex128 (f64) dof-major tensor."""
        import torch
        y = torch.empty_like(x)
        _check(lib().mgm_level_apply_prec(self.h, level, PREC[prec], C.c_void_p(_ptr(x)),
                                          C.c_void_p(_ptr(y)), x.shape[2]))
        return y

    def restrict(self, level: int, x, prec: str = "f64"):
        """y_c = P^H x; f64: complex128 vectors, f32: complex64 vectors with
        the FP16-stored P of a mixed hierarchy."""
        y = self._vec(level + 1, x.shape[2], x.dtype)
        if prec == "f64":
            _check(lib().mgm_restrict(self.h, level, C.c_void_p(_ptr(x)), C.c_void_p(_ptr(y)), x.shape[2]))
        else:
            _check(lib().mgm_restrict_prec(self.h, level, PREC[prec], C.c_void_p(_ptr(x)),
                                           C.c_void_p(_ptr(y)), x.shape[2]))
        return y

    def prolong(self, level: int, xc, prec: str = "f64"):
        """y = P x_c in precision prec (as restrict)."""
        y = self._vec(level, xc.shape[2], xc.dtype)
        if prec == "f64":
            _check(lib().mgm_prolong(self.h, level, C.c_void_p(_ptr(xc)), C.c_void_p(_ptr(y)), xc.shape[2]))
        else:
            _check(lib().mgm_prolong_prec(self.h, level, PREC[prec], C.c_void_p(_ptr(xc)),
                                          C.c_void_p(_ptr(y)), xc.shape[2]))
        return y

    def restrict_f16(self, level: int, x16, scale):
        """y_c = P^H (scale x16): x16 float16 pairs (dof, site, nrhs, 2) on the
        fine side, scale float64 (nrhs,); complex64 result (mixed hierarchies)."""
        import torch
        y = self._vec(level + 1, x16.shape[2], torch.complex64)
        _check(lib().mgm_restrict_f16(self.h, level, C.c_void_p(_ptr(x16)), C.c_void_p(_ptr(scale)),
                                      C.c_void_p(_ptr(y)), x16.shape[2]))
        return y

    def prolong_add_f16(self, level: int, xc, x16, scale):
        """y = scale x16 + P x_c: xc complex64 on the coarse side, x16 and scale
        as for restrict_f16; complex64 result."""
        import torch
        y = self._vec(level, xc.shape[2], torch.complex64)
        _check(lib().mgm_prolong_add_f16(self.h, level, C.c_void_p(_ptr(xc)), C.c_void_p(_ptr(x16)),
                                         C.c_void_p(_ptr(scale)), C.c_void_p(_ptr(y)), xc.shape[2]))
        return y

    def project_out(self, level: int, x):
        y = self._vec(level, x.shape[2])
        _check(lib().mgm_project_out(self.h, level, C.c_void_p(_ptr(x)), C.c_void_p(_ptr(y)), x.shape[2]))
        return y

    def solve(self, level: int, b, desc: SolveDesc | None = None, x=None, check: bool = True):
        desc = desc or solve_desc()
        if x is None:
            x = self._vec(level, b.shape[2])
        st = SolveStats()
        rc = lib().mgm_solve(self.h, level, C.byref(desc), C.c_void_p(_ptr(b)), C.c_void_p(_ptr(x)),
                             b.shape[2], C.byref(st))
        stats = {"iterations": st.iterations, "restarts": st.restarts, "fallbacks": st.fallbacks,
                 "max_rel_residual": st.max_rel_residual, "seconds": st.seconds, "status": rc}
        if check:
            _check(rc)
        return x, stats

    def estimate(self, observable: str, decomposition: str, nprobe, seed: int, batch=8,
                 first_probe: int = 0, solve: SolveDesc | None = None, samples: bool = True,
                 check: bool = True, deflation=None, noise="z4", probing: int = 0):
        """batch: an int, or a per-probe-group list (finest group first);
        deflation: a Deflation built on this hierarchy (decomposition
        "deflated")."""
        d = EstimateDesc()
        d.deflation = deflation.h if deflation is not None else None
        d.noise = NOISE[noise] if isinstance(noise, str) else int(noise)
        d.probing = int(probing)
        if not isinstance(batch, int):
            bl = list(batch) + [0] * (MAX_LEVELS - len(batch))
            d.batch_level[:] = bl[:MAX_LEVELS]
            batch = int(batch[0])
        d.observable = OBS[observable]
        d.decomposition = DEC[decomposition]
        npr = list(nprobe) + [0] * (MAX_LEVELS - len(nprobe))
        d.nprobe[:] = npr[:MAX_LEVELS]
        d.seed = seed
        d.first_probe = first_probe
        d.batch = batch
        d.solve = solve or solve_desc()
        sz = EstimateSizes()
        _check(lib().mgm_estimate_sizes_query(self.h, C.byref(d), C.byref(sz)))
        K = sz.ngamma * sz.T
        n = np.zeros(sz.nterms, dtype=np.int64)
        mean = np.zeros(sz.nterms * K * 2)
        var = np.zeros(sz.nterms * K)
        cost = np.zeros(sz.nterms)
        smp = np.zeros(max(1, sz.nsamples) * 2) if samples else None
        tm = np.zeros(K * 2)
        tv = np.zeros(K)
        r = EstimateResult()
        P = C.POINTER
        r.n = n.ctypes.data_as(P(C.c_int64))
        r.mean = mean.ctypes.data_as(P(C.c_double))
        r.var = var.ctypes.data_as(P(C.c_double))
        r.cost_s = cost.ctypes.data_as(P(C.c_double))
        r.samples = smp.ctypes.data_as(P(C.c_double)) if samples else None
        r.total_mean = tm.ctypes.data_as(P(C.c_double))
        r.total_var = tv.ctypes.data_as(P(C.c_double))
        rc = lib().mgm_estimate(self.h, C.byref(d), C.byref(r))
        if check:
            _check(rc)
        shape = (sz.nterms, sz.ngamma, sz.T)
        out = {"status": rc, "n": n, "mean": mean.view(np.complex128).reshape(shape),
               "var": var.reshape(shape), "cost_s": cost,
               "total_mean": tm.view(np.complex128).reshape(sz.ngamma, sz.T),
               "total_var": tv.reshape(sz.ngamma, sz.T),
               "stats": {"iterations": r.stats.iterations, "restarts": r.stats.restarts,
                         "max_rel_residual": r.stats.max_rel_residual, "seconds": r.stats.seconds,
                         "fallbacks": r.stats.fallbacks}}
        if samples:
            flat = smp[:2 * sz.nsamples].view(np.complex128)
            per, off = [], 0
            for q in range(sz.nterms):
                m = int(n[q]) * K
                per.append(flat[off:off + m].reshape(int(n[q]), sz.ngamma, sz.T))
                off += m
            out["samples"] = per
        return out

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.mgm_hierarchy_destroy(self.h)
            self.h = None


class Deflation:
    """Inexact deflation basis V of the hierarchy's fine operator (inverse
    block power on Gamma5 D) and its exact term tr(V^H D^-1 V)."""

    def __init__(self, hierarchy: Hierarchy, k: int, power_iters: int = 5, power_tol: float = 1e-6,
                 seed: int = 1, batch: int | None = None, solve: SolveDesc | None = None, check: bool = True):
        self.hier = hierarchy
        d = DeflationDesc()
        d.k, d.power_iters, d.power_tol, d.seed = k, power_iters, power_tol, seed
        d.batch = batch if batch is not None else min(k, hierarchy.desc.max_nrhs_level[0] or hierarchy.desc.max_nrhs)
        d.solve = solve or solve_desc()
        self.desc = d
        self.k = k
        nb = C.c_size_t()
        _check(lib().mgm_deflation_workspace_size(hierarchy.h, C.byref(d), C.byref(nb)))
        self.ws = _empty_ws(nb.value, hierarchy.ctx.device)
        h = C.c_void_p()
        rc = lib().mgm_deflation_create(hierarchy.h, C.byref(d), C.c_void_p(_ptr(self.ws)), self.ws.numel(),
                                        C.byref(h))
        self.status = rc
        if rc == 0 or rc == -4:
            self.h = h
        if check:
            _check(rc)

    def info(self) -> dict:
        tr = (C.c_double * 2)()
        a, b = C.c_double(), C.c_double()
        _check(lib().mgm_deflation_info(self.h, tr, C.byref(a), C.byref(b)))
        return {"exact_trace": complex(tr[0], tr[1]), "setup_s": a.value, "exact_s": b.value}

    def export(self) -> np.ndarray:
        """V as (k, sites, 12) complex128 (column j = basis vector j)."""
        s, d, n = self.hier.level_info(0)
        out = np.zeros((d, s, self.k), dtype=np.complex128)
        _check(lib().mgm_deflation_export(self.h, out.ctypes.data_as(C.c_void_p), out.nbytes))
        return from_dofmajor(out)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.mgm_deflation_destroy(self.h)
            self.h = None


def mlmc_allocate(var, cost, eps2: float) -> np.ndarray:
    var = np.ascontiguousarray(var, dtype=np.float64)
    cost = np.ascontiguousarray(cost, dtype=np.float64)
    out = np.zeros(len(var), dtype=np.int64)
    _check(lib().mgm_mlmc_allocate(len(var), var.ctypes.data_as(C.POINTER(C.c_double)),
                                   cost.ctypes.data_as(C.POINTER(C.c_double)), eps2,
                                   out.ctypes.data_as(C.POINTER(C.c_int64))))
    return out


class Net:
    """Gauge-covariant PTC network (the learned fine-level smoother) on the
    lattice of operator `op`.  widths = [4, c1, ..., 4]."""

    def __init__(self, op: Operator, widths=(4, 16, 16, 16, 4), seed: int = 1, max_nrhs: int = 8,
                 train_nrhs: int = 0, bf16_weights: bool = False):
        self.op = op
        self.ctx = op.ctx
        d = NetDesc()
        d.nlayers = len(widths) - 1
        for i, w in enumerate(widths):
            d.width[i] = int(w)
        d.seed = seed
        d.max_nrhs = max_nrhs
        d.train_nrhs = train_nrhs
        d.bf16_weights = 1 if bf16_weights else 0
        self.desc = d
        self.widths = list(widths)
        nb = C.c_size_t()
        _check(lib().mgm_net_workspace_size(op.h, C.byref(d), C.byref(nb)))
        self.ws = _empty_ws(nb.value, self.ctx.device)
        h = C.c_void_p()
        _check(lib().mgm_net_create(op.h, C.byref(d), C.c_void_p(_ptr(self.ws)), self.ws.numel(), C.byref(h)))
        self.h = h
        n = C.c_int64()
        _check(lib().mgm_net_num_weights(h, C.byref(n)))
        self.nweights = n.value

    def _split(self, flat: np.ndarray) -> list:
        out, off = [], 0
        for l in range(len(self.widths) - 1):
            ci, co = self.widths[l], self.widths[l + 1]
            k = 9 * co * ci
            out.append(flat[off:off + k].reshape(9, co, ci))
            off += k
        return out

    def bind(self, op: Operator):
        """Moves the network (weights and Adam state) to another operator of the same lattice."""
        _check(lib().mgm_net_bind(self.h, op.h))
        self.op = op

    def get_weights(self) -> list:
        w = np.empty(2 * self.nweights, dtype=np.float64)
        _check(lib().mgm_net_get_weights(self.h, w.ctypes.data_as(C.c_void_p)))
        return self._split(w.view(np.complex128))

    def save(self, path: str):
        """Writes the layer widths and FP64 weights to `path`."""
        _check(lib().mgm_net_save(self.h, os.fsencode(path)))

    def load(self, path: str):
        """Reads weights written by save() for a network of the same widths."""
        _check(lib().mgm_net_load(self.h, os.fsencode(path)))

    def set_weights(self, weights: list):
        flat = np.concatenate([np.asarray(W, dtype=np.complex128).ravel() for W in weights])
        if flat.size != self.nweights:
            raise ValueError("expected %d complex weights, got %d" % (self.nweights, flat.size))
        w = np.ascontiguousarray(flat).view(np.float64)
        _check(lib().mgm_net_set_weights(self.h, w.ctypes.data_as(C.c_void_p)))

    def apply(self, r, y=None):
        """y = N(r) for complex64 dof-major spinors (12, V, nrhs)."""
        import torch
        if y is None:
            y = torch.empty_like(r)
        _check(lib().mgm_net_apply(self.h, C.c_void_p(_ptr(r)), C.c_void_p(_ptr(y)), r.shape[2]))
        return y

    def loss_grad(self, r, e):
        """(loss, per-layer weight gradients) for complex64 pairs (12, V, n)."""
        loss = C.c_double()
        g = np.empty(2 * self.nweights, dtype=np.float64)
        _check(lib().mgm_net_loss_grad(self.h, C.c_void_p(_ptr(r)), C.c_void_p(_ptr(e)), r.shape[2],
                                       C.byref(loss), g.ctypes.data_as(C.c_void_p)))
        return loss.value, self._split(g.view(np.complex128))

    def train(self, hierarchy, steps: int = 100, lr: float = 1e-3, seed: int = 7, target_tol: float = 1e-8,
              beta1: float = 0.0, beta2: float = 0.0, eps: float = 0.0):
        d = TrainDesc()
        d.steps, d.lr, d.seed, d.target_tol = steps, lr, seed, target_tol
        d.beta1, d.beta2, d.eps = beta1, beta2, eps
        st = TrainStats()
        hist = np.zeros(steps, dtype=np.float64)
        _check(lib().mgm_net_train(self.h, hierarchy.h, C.byref(d), C.byref(st), hist.ctypes.data_as(C.c_void_p)))
        return {"loss_first": st.loss_first, "loss_last": st.loss_last, "steps": st.steps,
                "seconds": st.seconds, "history": hist}

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.mgm_net_destroy(self.h)
            self.h = None
