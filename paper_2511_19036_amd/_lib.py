"""ctypes binding of ``include/cmg.h`` (argument marshalling only).

Every computation runs inside ``libcmg.so``; this module only declares the C
signatures, converts torch device tensors to raw pointers and raises on
error codes.  There is no fallback: if the library is missing, :func:`load`
raises.
"""
from __future__ import annotations

import ctypes as C
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcmg.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "cmg.h")

OK, INVALID_ARG, UNSUPPORTED, OUT_OF_MEMORY, HIP, NONFINITE, NOT_CONVERGED = range(7)
POISSON, DIFFUSION = 0, 1
WJACOBI, RBGS = 0, 1
PLAIN_FP64, COMPACT_BFP = 0, 1
FP32, FP64 = 0, 1
SECTION_U, SECTION_R, SECTION_Y, SECTION_YPRE = 0, 1, 2, 3

STATUS_NAMES = {0: "CMG_OK", 1: "CMG_ERR_INVALID_ARG", 2: "CMG_ERR_UNSUPPORTED",
                3: "CMG_ERR_OUT_OF_MEMORY", 4: "CMG_ERR_HIP", 5: "CMG_ERR_NONFINITE",
                6: "CMG_ERR_NOT_CONVERGED"}


class cmg_problem(C.Structure):
    _fields_ = [("dim", C.c_int32), ("L", C.c_int32), ("coarsest", C.c_int32),
                ("op", C.c_int32), ("batch", C.c_int32)]


class cmg_opts(C.Structure):
    _fields_ = [("smoother", C.c_int32), ("omega", C.c_double), ("nu_pre", C.c_int32),
                ("nu_post", C.c_int32), ("ir_iters", C.c_int32), ("vcycles", C.c_int32),
                ("final_iters", C.c_int32), ("storage", C.c_int32), ("bfp_block", C.c_int32),
                ("bits_u", C.c_int32), ("bits_r", C.c_int32), ("bits_y", C.c_int32),
                ("inc_u", C.c_int32), ("inc_ry", C.c_int32), ("vcycle_prec", C.c_int32),
                ("keep_correction", C.c_int32)]


class cmg_stats(C.Structure):
    _fields_ = [("record", C.c_int32), ("count", C.c_int32), ("residual_norm", C.c_double * 256)]


class cmg_mem(C.Structure):
    _fields_ = [("sections", C.c_int64), ("coarse_fp64", C.c_int64), ("coarse_work", C.c_int64),
                ("fine_work", C.c_int64), ("kappa", C.c_int64), ("total", C.c_int64),
                ("interior_dofs", C.c_int64), ("logical_bits_per_dof", C.c_double)]


class CmgError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_P = C.c_void_p
_I32 = C.c_int32
_I64 = C.c_int64
_ST = C.c_int  # cmg_status

SIGNATURES = {
    "cmg_default_opts": (_ST, [C.POINTER(cmg_opts)]),
    "cmg_setup": (_ST, [C.POINTER(cmg_problem), C.POINTER(cmg_opts), _P, _P, C.POINTER(_P)]),
    "cmg_fmg_solve": (_ST, [_P, _P, _P, C.POINTER(cmg_stats)]),
    "cmg_vcycle": (_ST, [_P, _P, _P]),
    "cmg_adjoint_solve": (_ST, [_P, _P, _P, _P, _P]),
    "cmg_destroy": (_ST, [_P]),
    "cmg_last_error": (C.c_char_p, [_P]),
    "cmg_bfp_code_bytes": (_I64, [_I64, _I32, _I32]),
    "cmg_bfp_encode": (_ST, [_P, _I32, _I64, _I32, _I32, _P, _P, _P]),
    "cmg_bfp_decode": (_ST, [_P, _P, _I64, _I32, _I32, _P, _P]),
    "cmg_abfp_code_bytes": (_I64, [_I64, _I32]),
    "cmg_abfp_workspace_bytes": (_I64, [_I64]),
    "cmg_abfp_encode": (_ST, [_P, _I32, _I64, _I32, _P, _P, _P, _P, _P, _P]),
    "cmg_abfp_encode_noalloc": (_ST, [_P, _I32, _I64, _I32, _P, _P, _P, _P, _P]),
    "cmg_abfp_decode": (_ST, [_P, _P, _P, _P, _I64, _I32, _P, _P]),
    "cmg_section_info": (_ST, [_P, _I32, _I32, C.POINTER(_I64), C.POINTER(_I32), C.POINTER(_I32),
                               C.POINTER(_I64), C.POINTER(_I64)]),
    "cmg_export_section": (_ST, [_P, _I32, _I32, _P, _P]),
    "cmg_import_section": (_ST, [_P, _I32, _I32, _I32, _P, _P]),
    "cmg_fmg_enter_level": (_ST, [_P, _I32, _P]),
    "cmg_ir_residual": (_ST, [_P, _P]),
    "cmg_vcycle_correct": (_ST, [_P]),
    "cmg_up_sweep": (_ST, [_P, _I32, _P]),
    "cmg_decode_solution": (_ST, [_P, _P]),
    "cmg_memory_stats": (_ST, [_P, C.POINTER(cmg_mem)]),
    "cmg_timing_enable": (_ST, [_P, _I32, C.c_char_p]),
    "cmg_timing_count": (_ST, [_P, C.POINTER(_I32)]),
    "cmg_timing_entry": (_ST, [_P, _I32, C.c_char_p, _I32, C.POINTER(_I64), C.POINTER(C.c_double),
                               C.POINTER(C.c_double)]),
}

_lib = None


def header_symbols() -> list[str]:
    """Every function name declared in ``include/cmg.h``."""
    with open(HEADER) as fh:
        text = fh.read()
    return sorted(set(re.findall(r"^\s*(?:cmg_status|int64_t|const char\*)\s+(cmg_\w+)\s*\(", text, re.M)))


def load(path: str | None = None):
    """Load ``libcmg.so`` (or the build named by the environment variable
    ``CMG_LIBRARY``, e.g. the host-sanitized one) and declare its signatures
    (raises if absent)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or os.environ.get("CMG_LIBRARY") or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int, ctx=None):
    if status != OK:
        lib = load()
        msg = lib.cmg_last_error(ctx).decode(errors="replace")
        raise CmgError(status, msg)


def ptr(t) -> int | None:
    """Raw device pointer of a torch tensor (None for None)."""
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream
