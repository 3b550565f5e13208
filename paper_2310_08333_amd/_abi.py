"""ctypes mirror of include/genios.h and the library loader.

The loader raises if libgenios.so is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgenios.so")

# status codes
OK = 0
MAX_ITER = 1
WARN_PRECOND = 2
ERR_ARG = -1
ERR_SHAPE = -2
ERR_NUMERIC = -3
ERR_FACTOR = -4
ERR_DEVICE = -5
ERR_WORKSPACE = -6
ERR_UNSUPPORTED = -7

DT_F32, DT_BF16, DT_F64 = 0, 1, 2
PREC_F64, PREC_F32, PREC_BF16_REFINE, PREC_BF16_ONLY = 0, 1, 2, 3
OP_LASSO, OP_LOGREG, OP_NYSTROM, OP_BACKWARD, OP_MATVEC, OP_HVP, OP_HUBER, OP_BOXLS = range(8)

HIST_FIELDS = 10
HIST_NAMES = ("k", "r_p", "r_d", "r_kkt", "rho", "cg", "rtol", "phase", "time", "xnorm")

PRECISIONS = {"f64": PREC_F64, "f32": PREC_F32, "bf16_refine": PREC_BF16_REFINE,
              "bf16_only": PREC_BF16_ONLY}


class Matrix(C.Structure):
    _fields_ = [("m", C.c_int64), ("n", C.c_int64), ("lda", C.c_int64), ("batch", C.c_int64),
                ("stride_A", C.c_int64), ("hi_dtype", C.c_int32), ("reserved", C.c_int32),
                ("A_hi", C.c_void_p), ("A_bf16", C.c_void_p)]


class Opts(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("precision", C.c_int32),
                ("sigma", C.c_double), ("alpha", C.c_double), ("gamma", C.c_double),
                ("eps_abs", C.c_double), ("eps_rel", C.c_double),
                ("tau", C.c_double), ("mu", C.c_double),
                ("rho_update_every", C.c_int32), ("rho_update_until", C.c_int32),
                ("max_iter", C.c_int32), ("max_cg_iter", C.c_int32),
                ("cg_tol_floor", C.c_double),
                ("sketch_rank", C.c_int32), ("resketch_every", C.c_int32),
                ("precondition", C.c_int32), ("inexact", C.c_int32),
                ("switch_tol", C.c_double),
                ("stall_window", C.c_int32), ("rhs_relative", C.c_int32),
                ("seed", C.c_uint64),
                ("warm_start", C.c_int32), ("profile_kernels", C.c_int32),
                ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t),
                ("stream", C.c_void_p),
                ("history", C.POINTER(C.c_double)), ("history_cap", C.c_int32),
                ("termination", C.c_int32), ("gap_every", C.c_int32),
                ("eps_gap", C.c_double), ("lambda2", C.c_double),
                ("huber_delta", C.c_double), ("adaptive_sketch", C.c_int32),
                ("sketch_rank_init", C.c_int32), ("sketch_kappa", C.c_double),
                ("power_iters", C.c_int32), ("batch_mfma", C.c_int32),
                ("refine_cg_bf16", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("cg_iters", C.c_int32),
                ("phase_switch_iter", C.c_int32), ("resketches", C.c_int32),
                ("precond_rank", C.c_int32),
                ("obj", C.c_double), ("r_p", C.c_double), ("r_d", C.c_double),
                ("r_kkt", C.c_double), ("rho", C.c_double),
                ("t_setup", C.c_double), ("t_precond", C.c_double), ("t_solve", C.c_double),
                ("t_linsys", C.c_double), ("t_prox", C.c_double), ("t_total", C.c_double),
                ("t_to_target", C.c_double), ("t_matvec_n", C.c_double),
                ("t_matvec_t", C.c_double), ("n_matvec_n", C.c_int32),
                ("n_matvec_t", C.c_int32), ("bytes_matvec_n", C.c_int64),
                ("bytes_matvec_t", C.c_int64), ("t_hvp", C.c_double), ("n_hvp", C.c_int32),
                ("n_hvp_hi", C.c_int32), ("bytes_hvp", C.c_int64), ("t_hvp_hi", C.c_double),
                ("bytes_hvp_hi", C.c_int64), ("t_sketch_mc", C.c_double),
                ("flops_sketch_mc", C.c_int64), ("n_sketch_mc", C.c_int32),
                ("n_sketch_fma", C.c_int32), ("t_sketch_fma", C.c_double),
                ("flops_sketch_fma", C.c_int64), ("rel_gap", C.c_double),
                ("gap_primal", C.c_double), ("gap_dual", C.c_double),
                ("gap_checks", C.c_int32), ("n_hvp_tail", C.c_int32),
                ("subgrad_dist", C.c_double), ("sketch_err", C.c_double),
                ("kappa_bound", C.c_double), ("sketch_rounds", C.c_int32),
                ("n_hvp_mrhs", C.c_int32), ("t_hvp_mrhs", C.c_double),
                ("bytes_hvp_mrhs", C.c_int64), ("n_hvp_resized", C.c_int32),
                ("reserved3", C.c_int32), ("bf16_bound", C.c_double)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


EXPORTED = (
    "genios_default_opts", "genios_workspace_size", "genios_lasso_solve", "genios_logreg_solve",
    "genios_huber_solve", "genios_boxls_solve",
    "genios_nystrom_build", "genios_nystrom_apply", "genios_lasso_backward", "genios_matvec",
    "genios_hvp", "genios_hvp_noalloc",
    "genios_cast_bf16", "genios_stream_read", "genios_gaussian_matrix", "genios_admm_update", "genios_status_string",
    "genios_last_error", "genios_abi_struct_sizes",
)

_lib = None


def load(path: str | None = None):
    """Load libgenios.so once; raise if it is missing (build it with build())."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"{p} not found: the HIP library is required (run "
                          f"`python paper_2310_08333_amd/build.py`); there is no CPU fallback")
    lib = C.CDLL(p)
    P = C.POINTER
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    lib.genios_default_opts.argtypes = [P(Opts)]
    lib.genios_default_opts.restype = C.c_int
    lib.genios_workspace_size.argtypes = [C.c_int, P(Matrix), P(Opts)]
    lib.genios_workspace_size.restype = C.c_size_t
    for name in ("genios_lasso_solve", "genios_logreg_solve", "genios_huber_solve"):
        f = getattr(lib, name)
        f.argtypes = [P(Matrix), vp, P(dbl), dbl, P(Opts), vp, vp, vp, P(Info)]
        f.restype = C.c_int
    lib.genios_boxls_solve.argtypes = [P(Matrix), vp, vp, vp, dbl, P(Opts), vp, vp, vp, P(Info)]
    lib.genios_boxls_solve.restype = C.c_int
    lib.genios_nystrom_build.argtypes = [P(Matrix), vp, i32, vp, P(Opts), vp, vp, P(Info)]
    lib.genios_nystrom_build.restype = C.c_int
    lib.genios_nystrom_apply.argtypes = [i64, i32, i64, i32, vp, vp, dbl, vp, vp, P(Opts)]
    lib.genios_nystrom_apply.restype = C.c_int
    lib.genios_lasso_backward.argtypes = [P(Matrix), vp, vp, P(dbl), P(Opts), vp, P(dbl), P(Info)]
    lib.genios_lasso_backward.restype = C.c_int
    lib.genios_matvec.argtypes = [P(Matrix), i32, i32, vp, vp, P(Opts)]
    lib.genios_matvec.restype = C.c_int
    lib.genios_hvp.argtypes = [P(Matrix), i32, vp, vp, vp, P(Opts)]
    lib.genios_hvp.restype = C.c_int
    lib.genios_hvp_noalloc.argtypes = [P(Matrix), i32, vp, vp, vp, P(Opts)]
    lib.genios_hvp_noalloc.restype = C.c_int
    lib.genios_cast_bf16.argtypes = [vp, vp, i64, P(Opts)]
    lib.genios_cast_bf16.restype = C.c_int
    lib.genios_stream_read.argtypes = [vp, i64, C.c_int32, vp, P(C.c_double), P(Opts)]
    lib.genios_stream_read.restype = C.c_int
    lib.genios_gaussian_matrix.argtypes = [i64, i32, C.c_uint64, C.c_uint64, vp, P(Opts)]
    lib.genios_gaussian_matrix.restype = C.c_int
    lib.genios_admm_update.argtypes = [i64, i32, dbl, dbl, vp, vp, vp, P(dbl), P(Opts)]
    lib.genios_admm_update.restype = C.c_int
    lib.genios_status_string.argtypes = [C.c_int]
    lib.genios_status_string.restype = C.c_char_p
    lib.genios_last_error.argtypes = []
    lib.genios_last_error.restype = C.c_char_p
    lib.genios_abi_struct_sizes.argtypes = [P(C.c_size_t), P(C.c_size_t), P(C.c_size_t)]
    lib.genios_abi_struct_sizes.restype = None
    sizes = [C.c_size_t(), C.c_size_t(), C.c_size_t()]
    lib.genios_abi_struct_sizes(*[C.byref(s) for s in sizes])
    got = tuple(s.value for s in sizes)
    want = (C.sizeof(Matrix), C.sizeof(Opts), C.sizeof(Info))
    if got != want:
        raise ImportError(f"genios struct layout mismatch: library {got}, binding {want}")
    _lib = lib
    return lib


def default_opts() -> Opts:
    o = Opts()
    load().genios_default_opts(C.byref(o))
    return o


def last_error() -> str:
    return load().genios_last_error().decode()


def status_string(code: int) -> str:
    return load().genios_status_string(code).decode()


class GeniosError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where} failed with {code} ({status_string(code)}): {last_error()}")
