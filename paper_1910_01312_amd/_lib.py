"""ctypes binding of libssnalm.so (include/ssnalm.h): structures, function
prototypes and loading.  Argument marshalling only; all computation runs in
the HIP library.  Loading fails loudly if the library has not been built."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libssnalm.so")

OK, MAXITER, LINESEARCH_FAIL, WARMSTART_REJECTED = 0, 1, 2, 3
E_BADARG, E_NONFINITE, E_OOM, E_HIP = -1, -2, -3, -4
STATUS_NAMES = {0: "OK", 1: "MAXITER", 2: "LINESEARCH_FAIL", 3: "WARMSTART_REJECTED",
                -1: "E_BADARG", -2: "E_NONFINITE", -3: "E_OOM", -4: "E_HIP"}
DENSE, CSR = 0, 1
F64, F32, BF16 = 0, 1, 2
NEWTON_AUTO, NEWTON_CHOL, NEWTON_PCG = 0, 1, 2
PREC_FP64, PREC_MIXED = 0, 1


class Problem(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dtype", C.c_int32),
                ("n", C.c_int64), ("q", C.c_int64), ("nnz", C.c_int64),
                ("X", C.c_void_p), ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p),
                ("y", C.c_void_p), ("C", C.c_double), ("tol", C.c_double)]


class SvrProblem(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dtype", C.c_int32), ("n", C.c_int64), ("q", C.c_int64),
                ("X", C.c_void_p), ("y", C.c_void_p), ("C", C.c_double), ("eps", C.c_double),
                ("tol", C.c_double)]


class GeneralProblem(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dtype", C.c_int32), ("n", C.c_int64), ("q", C.c_int64),
                ("B", C.c_void_p), ("c", C.c_void_p), ("a", C.c_void_p), ("l", C.c_void_p),
                ("u", C.c_void_p), ("d", C.c_double), ("tol", C.c_double)]


KERNEL_RBF, KERNEL_LINEAR = 0, 1


class KernelProblem(C.Structure):
    _fields_ = [("kernel", C.c_int32), ("dtype", C.c_int32), ("n", C.c_int64), ("q", C.c_int64),
                ("X", C.c_void_p), ("y", C.c_void_p), ("C", C.c_double), ("alpha", C.c_double),
                ("tol", C.c_double)]


class Options(C.Structure):
    _fields_ = [("sigma0", C.c_double), ("rho", C.c_double), ("sigma_max", C.c_double),
                ("mu", C.c_double), ("ls_delta", C.c_double), ("tau", C.c_double),
                ("eta", C.c_double), ("eps_decay", C.c_double), ("floor_rel", C.c_double),
                ("max_outer", C.c_int32), ("max_inner", C.c_int32),
                ("max_backtracks", C.c_int32), ("newton", C.c_int32),
                ("precision", C.c_int32), ("max_cg", C.c_int32), ("verbose", C.c_int32),
                ("check_finite", C.c_int32), ("profile", C.c_int32),
                ("batch_graphs", C.c_int32), ("autotune", C.c_int32), ("lowrank", C.c_int32)]


class WsStats(C.Structure):
    _fields_ = [("rounds", C.c_int32), ("kept", C.c_int32), ("fallback", C.c_int32),
                ("pad_", C.c_int32), ("rkkt_full", C.c_double), ("t_reduced", C.c_double)]


class Info(C.Structure):
    _fields_ = [("rkkt", C.c_double), ("obj", C.c_double), ("b", C.c_double),
                ("gap", C.c_double), ("sigma", C.c_double), ("time_s", C.c_double),
                ("t_matvec", C.c_double), ("t_proj", C.c_double), ("t_newton", C.c_double),
                ("t_other", C.c_double),
                ("iters_outer", C.c_int32), ("iters_inner", C.c_int32),
                ("cg_iters", C.c_int32), ("proj_passes", C.c_int32), ("p", C.c_int32),
                ("n_sv", C.c_int32), ("ls_fail", C.c_int32), ("ls_trials", C.c_int32),
                ("grad_steps", C.c_int32), ("proj_capped", C.c_int32), ("status", C.c_int32),
                ("lowrank_steps", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class KStat(C.Structure):
    _fields_ = [("launches", C.c_int64), ("seconds", C.c_double), ("bytes", C.c_double),
                ("flops", C.c_double)]


K_AMUL, K_ATMUL, K_AMUL_J, K_ATMUL_J, K_PROJ, K_SYRK, K_CHOL, K_QCOLS, K_QJJ, K_COUNT = range(10)
K_NAMES = ["amul", "atmul", "amul_J", "atmul_J", "proj_pass", "syrk", "chol", "qcols", "qjj"]

EXPORTS = [
    "ssnalm_default_options", "ssnalm_create", "ssnalm_solve", "ssnalm_solve_batch",
    "ssnalm_destroy", "ssnalm_last_error", "ssnalm_op_amul", "ssnalm_op_atmul",
    "ssnalm_op_project", "ssnalm_op_newton", "ssnalm_op_linesearch_trial", "ssnalm_op_rkkt",
    "ssnalm_kernel_stats", "ssnalm_op_gram", "ssnalm_batch_kernel_stats",
    "ssnalm_mlp_param_count", "ssnalm_mlp_work_floats", "ssnalm_mlp_scratch_floats",
    "ssnalm_mlp_forward", "ssnalm_mlp_backward", "ssnalm_mlp_adam", "ssnalm_ws_features",
    "ssnalm_ws_x0", "ssnalm_ws_solve", "ssnalm_set_profile", "ssnalm_ws_labels",
    "ssnalm_project_noalloc", "ssnalm_noalloc_max_n", "ssnalm_noalloc_scratch_bytes",
    "ssnalm_rff_features", "ssnalm_nystroem_features", "ssnalm_create_svr",
    "ssnalm_create_general", "ssnalm_create_kernel", "ssnalm_op_kernel_newton",
]

_lib = None


def load(path: str | None = None):
    """Load the HIP library (once).  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"libssnalm.so not built ({p}); run paper_1910_01312_amd/build.py")
    lib = C.CDLL(p)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    lib.ssnalm_default_options.argtypes = [C.POINTER(Options)]
    lib.ssnalm_default_options.restype = None
    lib.ssnalm_create.argtypes = [C.POINTER(vp), C.POINTER(Problem), C.POINTER(Options), vp]
    lib.ssnalm_create.restype = i32
    lib.ssnalm_solve.argtypes = [vp, vp, vp, vp, C.POINTER(dbl), C.POINTER(Info)]
    lib.ssnalm_solve.restype = i32
    lib.ssnalm_solve_batch.argtypes = [i32, C.POINTER(Problem), C.POINTER(Options), vp,
                                       C.POINTER(vp), C.POINTER(vp), C.POINTER(Info)]
    lib.ssnalm_solve_batch.restype = i32
    lib.ssnalm_destroy.argtypes = [vp]
    lib.ssnalm_destroy.restype = None
    lib.ssnalm_last_error.argtypes = []
    lib.ssnalm_last_error.restype = C.c_char_p
    lib.ssnalm_op_amul.argtypes = [vp, vp, vp]
    lib.ssnalm_op_amul.restype = i32
    lib.ssnalm_op_atmul.argtypes = [vp, vp, vp]
    lib.ssnalm_op_atmul.restype = i32
    lib.ssnalm_op_project.argtypes = [vp, vp, vp, vp, C.POINTER(dbl), C.POINTER(i64),
                                      C.POINTER(i32)]
    lib.ssnalm_op_project.restype = i32
    lib.ssnalm_op_newton.argtypes = [vp, vp, vp, dbl, dbl, vp, C.POINTER(i32)]
    lib.ssnalm_op_newton.restype = i32
    lib.ssnalm_op_linesearch_trial.argtypes = [vp, vp, vp, dbl, dbl, dbl, C.POINTER(dbl),
                                               C.POINTER(dbl)]
    lib.ssnalm_op_linesearch_trial.restype = i32
    lib.ssnalm_op_rkkt.argtypes = [vp, vp, C.POINTER(dbl), C.POINTER(dbl)]
    lib.ssnalm_op_rkkt.restype = i32
    lib.ssnalm_op_gram.argtypes = [vp, vp, vp]
    lib.ssnalm_op_gram.restype = i32
    lib.ssnalm_kernel_stats.argtypes = [vp, i32, C.POINTER(KStat), i32]
    lib.ssnalm_kernel_stats.restype = i32
    lib.ssnalm_batch_kernel_stats.argtypes = [i32, C.POINTER(KStat)]
    lib.ssnalm_batch_kernel_stats.restype = i32
    for name in ("ssnalm_mlp_param_count", "ssnalm_mlp_work_floats", "ssnalm_mlp_scratch_floats"):
        getattr(lib, name).restype = i64
    lib.ssnalm_mlp_param_count.argtypes = []
    lib.ssnalm_mlp_work_floats.argtypes = [i64]
    lib.ssnalm_mlp_scratch_floats.argtypes = [i64]
    lib.ssnalm_mlp_forward.argtypes = [vp, vp, i64, vp, vp, vp]
    lib.ssnalm_mlp_forward.restype = i32
    lib.ssnalm_mlp_backward.argtypes = [vp, vp, i64, vp, vp, vp, vp, C.c_float, vp, vp, vp, vp]
    lib.ssnalm_mlp_backward.restype = i32
    lib.ssnalm_mlp_adam.argtypes = [vp, vp, vp, vp, i64, C.c_float, C.c_float, C.c_float,
                                    C.c_float, i32, vp]
    lib.ssnalm_mlp_adam.restype = i32
    lib.ssnalm_ws_features.argtypes = [vp, vp, vp]
    lib.ssnalm_ws_features.restype = i32
    lib.ssnalm_project_noalloc.argtypes = [vp, vp, i64, dbl, vp, vp, C.POINTER(dbl),
                                           C.POINTER(i64), vp]
    lib.ssnalm_project_noalloc.restype = i32
    lib.ssnalm_noalloc_max_n.argtypes = []
    lib.ssnalm_noalloc_max_n.restype = i64
    lib.ssnalm_noalloc_scratch_bytes.argtypes = []
    lib.ssnalm_noalloc_scratch_bytes.restype = i64
    lib.ssnalm_create_general.argtypes = [C.POINTER(vp), C.POINTER(GeneralProblem), C.POINTER(Options), vp]
    lib.ssnalm_create_general.restype = i32
    lib.ssnalm_create_svr.argtypes = [C.POINTER(vp), C.POINTER(SvrProblem), C.POINTER(Options), vp]
    lib.ssnalm_create_svr.restype = i32
    lib.ssnalm_rff_features.argtypes = [vp, i32, i64, i64, vp, i64, vp, i32, vp]
    lib.ssnalm_rff_features.restype = i32
    lib.ssnalm_nystroem_features.argtypes = [vp, i32, i64, i64, vp, i64, dbl, dbl, vp, i32, vp]
    lib.ssnalm_nystroem_features.restype = i32
    lib.ssnalm_ws_labels.argtypes = [vp, vp, vp, vp]
    lib.ssnalm_ws_labels.restype = i32
    lib.ssnalm_ws_x0.argtypes = [vp, vp, vp]
    lib.ssnalm_ws_x0.restype = i32
    lib.ssnalm_ws_solve.argtypes = [vp, vp, dbl, i32, vp, vp, C.POINTER(Info), C.POINTER(WsStats)]
    lib.ssnalm_ws_solve.restype = i32
    lib.ssnalm_create_kernel.argtypes = [C.POINTER(vp), C.POINTER(KernelProblem), C.POINTER(Options), vp]
    lib.ssnalm_create_kernel.restype = i32
    lib.ssnalm_op_kernel_newton.argtypes = [vp, vp, vp, dbl, dbl, vp, vp, C.POINTER(dbl), C.POINTER(i32)]
    lib.ssnalm_op_kernel_newton.restype = i32
    lib.ssnalm_set_profile.argtypes = [vp, i32]
    lib.ssnalm_set_profile.restype = i32
    _lib = lib
    return lib


class SsnalmError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = load().ssnalm_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status: int, where: str) -> int:
    if status < 0:
        raise SsnalmError(status, where)
    return status


def default_options() -> Options:
    o = Options()
    load().ssnalm_default_options(C.byref(o))
    return o
