"""Compact (linear-storage) multigrid on AMD MI355X.

Python face of ``libcmg.so`` (C ABI in ``include/cmg.h``).  PyTorch supplies
device memory and the stream; every step of the solver runs in the HIP
library.  The main entry points:

* :class:`Solver` — one problem shape; ``solve(f)``, ``vcycle(r)``,
  ``adjoint(u, dJdu)``, section export/import and stepwise driving;
* :func:`bfp_encode` / :func:`bfp_decode` — the block floating point codec;
* :class:`paper_2511_19036_amd.autograd.CMGSolve` — differentiable solve.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import CmgError, load  # noqa: F401

__all__ = ["Solver", "bfp_encode", "bfp_decode", "bfp_code_bytes", "abfp_encode", "abfp_encode_noalloc", "abfp_decode",
           "abfp_workspace",
           "CmgError", "load", "options"]

_SMOOTHERS = {"wjacobi": _lib.WJACOBI, "rbgs": _lib.RBGS}
_OPS = {"poisson": _lib.POISSON, "diffusion": _lib.DIFFUSION}
_STORAGE = {"plain": _lib.PLAIN_FP64, "compact": _lib.COMPACT_BFP}
_PREC = {"fp32": _lib.FP32, "fp64": _lib.FP64}
_WHICH = {"u": _lib.SECTION_U, "r": _lib.SECTION_R, "y": _lib.SECTION_Y, "ypre": _lib.SECTION_YPRE}


def options(**kw) -> _lib.cmg_opts:
    """A ``cmg_opts`` from keyword arguments on top of the library defaults.

    Keys: smoother ("rbgs" | "wjacobi"), omega, nu_pre, nu_post, ir_iters,
    final_iters, storage ("compact" | "plain"), bfp_block, bits (sets
    bits_u, bits_r, bits_y), bits_u, bits_r, bits_y, inc_u, inc_ry,
    vcycle_prec ("fp32" | "fp64"), keep_correction (bool: keep the "y" and
    "ypre" sections for export).
    """
    lib = load()
    o = _lib.cmg_opts()
    _lib.check(lib.cmg_default_opts(C.byref(o)))
    kw = dict(kw)
    if "bits" in kw:
        b = kw.pop("bits")
        o.bits_u = o.bits_r = o.bits_y = int(b)
    for k, v in kw.items():
        if k == "smoother":
            v = _SMOOTHERS[v] if isinstance(v, str) else v
        elif k == "storage":
            v = _STORAGE[v] if isinstance(v, str) else v
        elif k == "vcycle_prec":
            v = _PREC[v] if isinstance(v, str) else v
        elif k == "keep_correction":
            v = int(bool(v))
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


class Solver:
    """A solver context for one problem shape (``cmg_setup`` .. ``cmg_destroy``).

    ``kappa``: float64 CUDA tensor of ``(2**L)**dim`` cells for diffusion.
    Arrays passed to the methods are contiguous float64 CUDA tensors of shape
    ``(batch, N, ..., N)`` or ``(N, ..., N)`` with ``N = 2**L + 1``.
    """

    def __init__(self, dim: int, L: int, op: str = "poisson", kappa=None, batch: int = 1,
                 coarsest: int = 1, stream=None, **opts):
        import torch
        self.lib = load()
        self.dim, self.L, self.batch = dim, L, batch
        self.N = (1 << L) + 1
        self.op = op
        self.problem = _lib.cmg_problem(dim, L, coarsest, _OPS[op], batch)
        self.opts = options(**opts)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._kappa = kappa
        ctx = C.c_void_p()
        st = self.lib.cmg_setup(C.byref(self.problem), C.byref(self.opts),
                                _lib.ptr(kappa), self.stream.cuda_stream, C.byref(ctx))
        if st != _lib.OK:
            raise CmgError(st, self.lib.cmg_last_error(None).decode())
        self.ctx = ctx

    # ------------------------------------------------------------ lifecycle
    def close(self):
        if getattr(self, "ctx", None):
            self.lib.cmg_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, status):
        _lib.check(status, self.ctx)

    def _node_shape(self, level=None):
        n = ((1 << (self.L if level is None else level)) + 1)
        return (n,) * self.dim

    def _nodes(self, t, name):
        """Validate a node tensor before its pointer crosses the C ABI."""
        import torch
        if t is None or not t.is_cuda or t.dtype != torch.float64:
            raise ValueError(f"{name} must be a float64 CUDA tensor")
        if t.numel() != self.batch * self.N ** self.dim:
            raise ValueError(f"{name} must hold batch * N**dim = {self.batch * self.N ** self.dim} values")
        return t.contiguous()

    def _out(self, like=None):
        import torch
        return torch.empty((self.batch,) + self._node_shape(), dtype=torch.float64, device="cuda")

    # ------------------------------------------------------------ solves
    def solve(self, f, u=None, record=False):
        """``cmg_fmg_solve``; returns ``u`` (and the residual norms if ``record``)."""
        f = self._nodes(f, "f")
        out = self._nodes(u, "u") if u is not None else self._out().reshape(f.shape)
        st = _lib.cmg_stats()
        st.record = 1 if record else 0
        self._check(self.lib.cmg_fmg_solve(self.ctx, _lib.ptr(f), _lib.ptr(out), C.byref(st)))
        if record:
            return out, [st.residual_norm[i] for i in range(st.count)]
        return out

    def vcycle(self, r, y=None):
        r = self._nodes(r, "r")
        out = self._nodes(y, "y") if y is not None else self._out().reshape(r.shape)
        self._check(self.lib.cmg_vcycle(self.ctx, _lib.ptr(r), _lib.ptr(out)))
        return out

    def adjoint(self, u, dJdu, want_grad=True):
        """``cmg_adjoint_solve``; returns ``(lambda, grad_kappa or None)``."""
        import torch
        u, dJdu = self._nodes(u, "u"), self._nodes(dJdu, "dJdu")
        lam = torch.empty_like(dJdu)
        grad = None
        if want_grad and self.op == "diffusion":
            grad = torch.empty(((1 << self.L),) * self.dim, dtype=torch.float64, device="cuda")
        self._check(self.lib.cmg_adjoint_solve(self.ctx, _lib.ptr(u), _lib.ptr(dJdu), _lib.ptr(lam),
                                               _lib.ptr(grad)))
        return lam, grad

    # ------------------------------------------------------------ stepwise
    def _single(self, t, name):
        """Validate one node array (N**dim values) for the stepwise calls."""
        import torch
        if t is None or not t.is_cuda or t.dtype != torch.float64 or t.numel() != self.N ** self.dim:
            raise ValueError(f"{name} must be a float64 CUDA tensor of N**dim values")
        return t.contiguous()

    def enter_level(self, level, f):
        self._check(self.lib.cmg_fmg_enter_level(self.ctx, level, _lib.ptr(self._single(f, "f"))))

    def ir_residual(self, f):
        self._check(self.lib.cmg_ir_residual(self.ctx, _lib.ptr(self._single(f, "f"))))

    def vcycle_correct(self):
        self._check(self.lib.cmg_vcycle_correct(self.ctx))

    def up_sweep(self, level, e_coarse):
        """``cmg_up_sweep``: one level's up sweep and correction from the
        current sections and a given coarse correction ``e_coarse`` (CUDA
        tensor of ``(2**(level-1))**dim`` values in the V-cycle type)."""
        import torch
        want = torch.float32 if self.opts.vcycle_prec == _lib.FP32 else torch.float64
        n = 1 << (level - 1)
        if e_coarse is None or not e_coarse.is_cuda or e_coarse.dtype != want or e_coarse.numel() != n ** self.dim:
            raise ValueError(f"e_coarse must be a {want} CUDA tensor of {n ** self.dim} values")
        self._check(self.lib.cmg_up_sweep(self.ctx, level, _lib.ptr(e_coarse.contiguous())))

    def decode_solution(self, level):
        import torch
        u = torch.empty(self._node_shape(level), dtype=torch.float64, device="cuda")
        self._check(self.lib.cmg_decode_solution(self.ctx, _lib.ptr(u)))
        return u

    # ------------------------------------------------------------ sections
    def section_info(self, which, level):
        n, w, cb, nbytes, nb = C.c_int64(), C.c_int32(), C.c_int32(), C.c_int64(), C.c_int64()
        self._check(self.lib.cmg_section_info(self.ctx, _WHICH[which], level, C.byref(n), C.byref(w),
                                              C.byref(cb), C.byref(nbytes), C.byref(nb)))
        return dict(n=n.value, bits=w.value, container_bits=cb.value, code_bytes=nbytes.value,
                    n_blocks=nb.value)

    def export_section(self, which, level):
        """Returns ``(codes: bytes-like uint8 array, exps: int16 array, bits)``."""
        info = self.section_info(which, level)
        codes = np.zeros(info["code_bytes"], dtype=np.uint8)
        exps = np.zeros(info["n_blocks"], dtype=np.int16)
        self._check(self.lib.cmg_export_section(self.ctx, _WHICH[which], level,
                                                codes.ctypes.data_as(C.c_void_p),
                                                exps.ctypes.data_as(C.c_void_p)))
        return codes, exps, info["bits"]

    def import_section(self, which, level, bits, codes, exps):
        info = self.section_info(which, level)
        codes = np.ascontiguousarray(codes, dtype=np.uint8)
        exps = np.ascontiguousarray(exps, dtype=np.int16)
        if codes.size != info["code_bytes"] or exps.size != info["n_blocks"]:
            raise ValueError("section size mismatch")
        self._check(self.lib.cmg_import_section(self.ctx, _WHICH[which], level, bits,
                                                codes.ctypes.data_as(C.c_void_p),
                                                exps.ctypes.data_as(C.c_void_p)))

    def timing(self, enable: bool = True, kernel: str | None = None):
        """Start (clearing totals) or stop per-kernel event timing."""
        self._check(self.lib.cmg_timing_enable(self.ctx, 1 if enable else 0,
                                               kernel.encode() if kernel else None))

    def timing_report(self) -> list[dict]:
        """Per-kernel launches, total ms and total algorithmic bytes."""
        cnt = C.c_int32()
        self._check(self.lib.cmg_timing_count(self.ctx, C.byref(cnt)))
        out = []
        for i in range(cnt.value):
            name = C.create_string_buffer(128)
            n, ms, b = C.c_int64(), C.c_double(), C.c_double()
            self._check(self.lib.cmg_timing_entry(self.ctx, i, name, 128, C.byref(n), C.byref(ms), C.byref(b)))
            out.append(dict(kernel=name.value.decode(), launches=n.value, ms=ms.value, bytes=b.value))
        return sorted(out, key=lambda r: -r["ms"])

    def memory_stats(self) -> dict:
        m = _lib.cmg_mem()
        self._check(self.lib.cmg_memory_stats(self.ctx, C.byref(m)))
        return {k: getattr(m, k) for k, _ in _lib.cmg_mem._fields_}


# ---------------------------------------------------------------- codec
def bfp_code_bytes(n: int, block: int, bits: int) -> int:
    return int(load().cmg_bfp_code_bytes(n, block, bits))


def bfp_encode(x, block: int, bits: int, stream=None):
    """Encode a float32/float64 CUDA tensor; returns ``(codes uint8, exps int16)``."""
    import torch
    lib = load()
    x = x.contiguous()
    n = x.numel()
    codes = torch.empty(max(bfp_code_bytes(n, block, bits), 1), dtype=torch.uint8, device=x.device)
    exps = torch.empty(max((n + block - 1) // block, 1), dtype=torch.int16, device=x.device)
    _lib.check(lib.cmg_bfp_encode(_lib.ptr(x), 1 if x.dtype == torch.float64 else 0, n, block, bits,
                                  _lib.ptr(codes), _lib.ptr(exps), _lib.stream_ptr(stream)))
    return codes, exps


def bfp_decode(codes, exps, n: int, block: int, bits: int, stream=None):
    import torch
    lib = load()
    x = torch.empty(n, dtype=torch.float64, device=codes.device)
    _lib.check(lib.cmg_bfp_decode(_lib.ptr(codes), _lib.ptr(exps), n, block, bits, _lib.ptr(x),
                                  _lib.stream_ptr(stream)))
    return x


# ------------------------------------------------------- adaptive codec
def abfp_workspace(n: int, device="cuda"):
    """Device workspace for one adaptive encode of ``n`` values."""
    import torch
    return torch.empty(int(load().cmg_abfp_workspace_bytes(n)), dtype=torch.uint8, device=device)


def abfp_encode(x, bits: int, stream=None, workspace=None):
    """Adaptive-exponent BFP encode of a float32/float64 CUDA tensor (Sec. 6.1.3).

    Returns ``(codes uint8, starts int64[bits], exps int16[bits], nblocks
    int32[1])``, all on the device; ``nblocks`` holds the kept block count
    (-1: non-finite input).  Asynchronous: nothing is synchronised here."""
    import torch
    lib = load()
    x = x.contiguous()
    n = x.numel()
    dev = x.device
    codes = torch.empty(max(int(lib.cmg_abfp_code_bytes(n, bits)), 16), dtype=torch.uint8, device=dev)
    starts = torch.empty(bits, dtype=torch.int64, device=dev)
    exps = torch.empty(bits, dtype=torch.int16, device=dev)
    nblocks = torch.empty(1, dtype=torch.int32, device=dev)
    if workspace is None:
        workspace = abfp_workspace(n, dev)
    _lib.check(lib.cmg_abfp_encode(_lib.ptr(x), 1 if x.dtype == torch.float64 else 0, n, bits, _lib.ptr(codes),
                                   _lib.ptr(starts), _lib.ptr(exps), _lib.ptr(nblocks), _lib.ptr(workspace),
                                   _lib.stream_ptr(stream)))
    return codes, starts, exps, nblocks


def abfp_encode_noalloc(x, bits: int, codes, starts, exps, nblocks, stream=None):
    """``cmg_abfp_encode_noalloc``: :func:`abfp_encode` into caller-given
    output tensors, with the library's static workspace (nothing is
    allocated; at most 2**31 values)."""
    import torch
    lib = load()
    x = x.contiguous()
    _lib.check(lib.cmg_abfp_encode_noalloc(_lib.ptr(x), 1 if x.dtype == torch.float64 else 0, x.numel(), bits,
                                           _lib.ptr(codes), _lib.ptr(starts), _lib.ptr(exps), _lib.ptr(nblocks),
                                           _lib.stream_ptr(stream)))


def abfp_decode(codes, starts, exps, nblocks, n: int, bits: int, stream=None):
    """Float64 values of an adaptive encode's outputs."""
    import torch
    lib = load()
    x = torch.empty(n, dtype=torch.float64, device=codes.device)
    _lib.check(lib.cmg_abfp_decode(_lib.ptr(codes), _lib.ptr(starts), _lib.ptr(exps), _lib.ptr(nblocks), n, bits,
                                   _lib.ptr(x), _lib.stream_ptr(stream)))
    return x
