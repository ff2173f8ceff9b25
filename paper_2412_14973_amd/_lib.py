"""ctypes view of the C ABI in include/tlrmdd.h (argument marshalling only).

The library must be built (``python -m paper_2412_14973_amd.build`` or
``__graft_entry__.build()``); loading fails loudly when it is missing. torch
is imported first so the library binds to the HIP runtime torch already
loaded (one runtime per process).
"""
import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime the library links)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libtlrmdd.so")

OK, INVALID_ARGUMENT, WORKSPACE, HIP_ERROR, NONFINITE, UNSUPPORTED, NOT_CONVERGED = 0, 1, 2, 3, 4, 5, 6
FP32, BF16X3, FP32_3M = 0, 1, 2
LBFGS, GD = 0, 1
OP_FORWARD, OP_GRAD, OP_SOLVE = 0, 1, 2


class TLRMDDError(RuntimeError):
    def __init__(self, status, func, detail):
        super().__init__(f"{func} failed with status {status}: {detail}")
        self.status = status


class c_layout(ctypes.Structure):
    _fields_ = [("nr", ctypes.c_int64), ("ns", ctypes.c_int64), ("ntiles", ctypes.c_int32),
                ("tile_size", ctypes.POINTER(ctypes.c_int32)),
                ("rank_off", ctypes.POINTER(ctypes.c_int32)),
                ("rank_diag", ctypes.POINTER(ctypes.c_int32))]


class c_opts(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("optimizer", ctypes.c_int32), ("lbfgs_m", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("lam", ctypes.c_double), ("resid_refresh", ctypes.c_int32),
                ("streams", ctypes.c_int32), ("line_products", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class c_kernel_stats(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double), ("launches", ctypes.c_int64), ("cflops", ctypes.c_double),
                ("flops", ctypes.c_double), ("bytes", ctypes.c_double), ("flop_dtype", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class c_admm_opts(ctypes.Structure):
    _fields_ = [("inner", c_opts), ("nstages", ctypes.c_int32), ("outer", ctypes.c_int32),
                ("lambdas", ctypes.POINTER(ctypes.c_double)), ("rho", ctypes.c_double)]


_lib = None

_SIGS = {
    "tlrmdd_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "tlrmdd_last_error": (ctypes.c_char_p, []),
    "tlrmdd_theta_size": (ctypes.c_int64, [ctypes.POINTER(c_layout)]),
    "tlrmdd_plan_create": (ctypes.c_int, [ctypes.POINTER(c_layout), ctypes.POINTER(ctypes.c_void_p)]),
    "tlrmdd_plan_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "tlrmdd_workspace_bytes": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(c_opts),
                                              ctypes.POINTER(ctypes.c_size_t)]),
    "tlrmdd_forward": (ctypes.c_int, [ctypes.c_void_p] * 7 + [ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t,
                                                                ctypes.c_void_p]),
    "tlrmdd_grad": (ctypes.c_int, [ctypes.c_void_p] * 6 + [ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t,
                                                             ctypes.c_void_p]),
    "tlrmdd_grad_noalloc": (ctypes.c_int, [ctypes.c_void_p] * 6 + [ctypes.c_int, ctypes.c_void_p]),
    "tlrmdd_solve": (ctypes.c_int, [ctypes.c_void_p] * 4 + [ctypes.POINTER(c_opts), ctypes.c_void_p,
                                                              ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "tlrmdd_line_form": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(c_opts), ctypes.POINTER(ctypes.c_int),
                                        ctypes.POINTER(ctypes.c_int)]),
    "tlrmdd_workspace_bytes_batched": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_void_p),
                                                      ctypes.POINTER(c_opts), ctypes.POINTER(ctypes.c_size_t)]),
    "tlrmdd_solve_batched": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_void_p),
                                            ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                                            ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(c_opts),
                                            ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p, ctypes.c_size_t,
                                            ctypes.c_void_p]),
    "hilbert_order": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]),
    "tlrmdd_permute_columns": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                              ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]),
    "tlrmdd_adjoint": (ctypes.c_int, [ctypes.c_void_p] * 4 + [ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t,
                                                                ctypes.c_void_p]),
    "tlrmdd_workspace_bytes_admm": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_void_p),
                                                   ctypes.POINTER(c_admm_opts), ctypes.POINTER(ctypes.c_size_t)]),
    "tlrmdd_admm": (ctypes.c_int, [ctypes.c_void_p] * 4 + [ctypes.POINTER(c_admm_opts), ctypes.c_void_p,
                                                          ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "tlrmdd_admm_batched": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_void_p),
                                           ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                                           ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(c_admm_opts),
                                           ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p, ctypes.c_size_t,
                                           ctypes.c_void_p]),
    "tlrmdd_workspace_bytes_ranks": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]),
    "tlrmdd_tile_ranks": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                         ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "tlrmdd_choose_layout": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int32,
                                            ctypes.c_double, ctypes.POINTER(ctypes.c_int32), ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                            ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "tlrmdd_workspace_bytes_warm": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)]),
    "tlrmdd_warm_start": (ctypes.c_int, [ctypes.c_void_p] * 4 + [ctypes.c_size_t, ctypes.c_void_p]),
    "tlrmdd_workspace_bytes_tlr": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)]),
    "tlrmdd_forward_tlr": (ctypes.c_int, [ctypes.c_void_p] * 7 + [ctypes.c_size_t, ctypes.c_void_p]),
    "tlrmdd_timing_begin": (ctypes.c_int, []),
    "tlrmdd_timing_begin_kinds": (ctypes.c_int, [ctypes.c_uint32]),
    "tlrmdd_timing_end": (ctypes.c_int, [ctypes.c_void_p]),
    "tlrmdd_graph_begin": (ctypes.c_int, [ctypes.c_void_p]),
    "tlrmdd_graph_end": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "tlrmdd_graph_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "tlrmdd_graph_destroy": (ctypes.c_int, [ctypes.c_void_p]),
}
(K_GEMM_RESID, K_GEMM_ADJOINT, K_GEMM_LINE, K_ASSEMBLE, K_ASSEMBLE_DIR, K_GRAD, K_LINE_PACK, K_LINE_TILE,
 K_GRAD_TILE, K_RESID_TILE, K_STAGE, K_PERMUTE, K_GRAM, K_COMBINE, K_THETA_UPDATE, K_RESID_UPDATE,
 K_NKINDS) = range(17)
KIND_NAMES = ("gemm_resid", "gemm_adjoint", "gemm_line", "assemble", "assemble_dir", "grad", "line_pack", "line_tile",
              "grad_tile", "resid_tile", "stage", "permute", "gram", "combine", "theta_update", "resid_update")
DT_NONE, DT_FP32, DT_BF16, DT_MIXED = -1, 0, 1, 2

EXPORTS = tuple(_SIGS)


def load():
    """Load the built library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"TLR-MDD HIP library not built: {LIB_PATH} is missing "
                           "(run __graft_entry__.build() or python -m paper_2412_14973_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status, func):
    if status != OK:
        lib = load()
        detail = lib.tlrmdd_last_error().decode() or lib.tlrmdd_status_string(status).decode()
        raise TLRMDDError(status, func, detail)
