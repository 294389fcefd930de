"""ctypes declarations of the C ABI in include/amm.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libamm.so")

AMM_OK = 0
STATUS_NAMES = {0: "AMM_OK", 1: "AMM_EINVAL", 2: "AMM_ESHAPE", 3: "AMM_EUNSUPPORTED",
                4: "AMM_ENOMEM", 5: "AMM_EDEVICE", 6: "AMM_ESTATE"}

AMM_CIRCULANT = 1
AMM_TSVD = 2
AMM_SPARSE = 4
AMM_SFFT = 8


class AmmOpts(C.Structure):
    _fields_ = [("sparse_frac", C.c_double), ("sparse_nnz", C.c_int64),
                ("oversample", C.c_int), ("power_iters", C.c_int),
                ("seed", C.c_uint64), ("keep_residual", C.c_int), ("spectral_fp16", C.c_int)]


class AmmDecInfo(C.Structure):
    _fields_ = [("kind", C.c_int), ("m", C.c_int64), ("n", C.c_int64), ("K", C.c_int),
                ("K_eff", C.c_int), ("nnz", C.c_int64), ("has_residual", C.c_int),
                ("norm_A", C.c_double), ("norm_residual", C.c_double), ("blocks", C.c_int),
                ("spectral_fp16", C.c_int), ("mu", C.c_double), ("sigma_next", C.c_double)]


AMM_ENTRIES_SIGNED = 0
AMM_ENTRIES_UNSIGNED_UNIFORM = 1


class AmmErrorEstimate(C.Structure):
    _fields_ = [("norm_A", C.c_double), ("norm_B", C.c_double), ("norm_dA", C.c_double),
                ("norm_dB", C.c_double), ("norm_M", C.c_double), ("prior", C.c_double),
                ("posterior", C.c_double), ("svd_bound", C.c_double), ("cd_estimate", C.c_double),
                ("spec_dA", C.c_double), ("spec_dB", C.c_double), ("mu_A", C.c_double), ("mu_B", C.c_double)]


AMM_F32, AMM_BF16, AMM_F16 = 0, 1, 2


class AmmMatrix(C.Structure):
    _fields_ = [("data", C.c_void_p), ("rows", C.c_int64), ("cols", C.c_int64), ("ld", C.c_int64),
                ("dtype", C.c_int)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_int, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_int, C.c_void_p)


class AmmAllocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", C.c_void_p)]


# name -> (restype, argtypes); every pointer is a plain void* / typed pointer
SIGNATURES = {
    "amm_opts_default": (None, [C.POINTER(AmmOpts)]),
    "amm_last_error": (C.c_char_p, []),
    "amm_ctx_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int]),
    "amm_ctx_create_with_allocator": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.POINTER(AmmAllocator)]),
    "amm_ctx_destroy": (None, [C.c_void_p]),
    "amm_ctx_set_timing": (C.c_int, [C.c_void_p, C.c_int]),
    "amm_ctx_set_debug": (C.c_int, [C.c_void_p, C.c_int]),
    "amm_ctx_set_tune_cache": (C.c_int, [C.c_void_p, C.c_char_p]),
    "amm_batch_tuned_from_cache": (C.c_int, [C.c_void_p, C.POINTER(C.c_int)]),
    "amm_ctx_timings": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int,
                                  C.POINTER(C.c_int)]),
    "amm_decompose": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_int, C.c_int,
                                C.POINTER(AmmOpts), C.c_void_p, C.POINTER(C.c_void_p)]),
    "amm_dec_import_circulant": (C.c_int, [C.c_void_p, C.c_int64, C.c_int, C.c_void_p, C.c_void_p,
                                           C.c_void_p, C.c_double, C.c_double, C.POINTER(C.c_void_p)]),
    "amm_dec_import_tsvd": (C.c_int, [C.c_void_p, C.c_int64, C.c_int64, C.c_int, C.c_void_p,
                                      C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p)]),
    "amm_dec_import_sparse": (C.c_int, [C.c_void_p, C.c_int64, C.c_int64, C.c_int64, C.c_void_p,
                                        C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.POINTER(C.c_void_p)]),
    "amm_dec_block": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_void_p)]),
    "amm_dec_query": (C.c_int, [C.c_void_p, C.POINTER(AmmDecInfo)]),
    "amm_dec_frequencies": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.POINTER(C.c_int)]),
    "amm_dec_energies": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64]),
    "amm_dec_circulant_lists": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64]),
    "amm_dec_tsvd_factors": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "amm_dec_sparse_part": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "amm_dec_destroy": (None, [C.c_void_p]),
    "amm_dec_export": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_size_t)]),
    "amm_dec_import": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(C.c_void_p)]),
    "amm_approx_matmul": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                    C.c_int64, C.c_void_p, C.c_void_p]),
    "amm_approx_matmul_strided": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                            C.c_int64, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p]),
    "amm_approx_matmul_static": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                           C.c_int64, C.c_void_p, C.c_void_p]),
    "amm_batch_plan_create": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.POINTER(C.c_void_p)]),
    "amm_batch_plan_create_bf16": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.POINTER(C.c_void_p)]),
    "amm_batch_run": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p]),
    "amm_batch_info": (C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int),
                                 C.POINTER(C.c_double)]),
    "amm_batch_plan_destroy": (None, [C.c_void_p]),
    "amm_batch_circulant_set_mode": (C.c_int, [C.c_void_p, C.c_int]),
    "amm_batch_circulant_schedule": (C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                               C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "amm_approx_matmul_backward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                             C.c_void_p, C.c_void_p, C.c_void_p]),
    "amm_approx_matmul_ex": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(AmmMatrix),
                                       C.POINTER(AmmMatrix), C.c_void_p]),
    "amm_approx_matmul_backward_ex": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(AmmMatrix), C.POINTER(AmmMatrix),
                                                C.POINTER(AmmMatrix), C.POINTER(AmmMatrix), C.c_void_p]),
    "amm_estimate_error": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int64,
                                     C.c_int, C.c_void_p, C.POINTER(AmmErrorEstimate)]),
    "amm_estimate_sketch": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                      C.c_int64, C.c_int64, C.c_int64, C.c_void_p, C.POINTER(C.c_double)]),
    "amm_choose_rank": (C.c_int, [C.c_void_p, C.c_void_p, C.c_double, C.c_int, C.POINTER(C.c_int)]),
    "amm_dec_set_sigma_next": (C.c_int, [C.c_void_p, C.c_double]),
    "amm_dec_set_spectral_fp16": (C.c_int, [C.c_void_p, C.c_int]),
}

_lib = None


class AmmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def load(path: str = LIB_PATH):
    """Load libamm.so (raises if it is missing: there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2504_19308_amd.build`")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int):
    if status != AMM_OK:
        msg = load().amm_last_error()
        raise AmmError(status, msg.decode() if msg else "")
