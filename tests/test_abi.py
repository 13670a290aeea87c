"""C ABI contract checks that need no GPU: the library loads, exports every
function ``include/cmg.h`` declares, and rejects invalid arguments before
touching the device."""
import ctypes as C

import pytest

from paper_2511_19036_amd import _lib


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def test_every_header_symbol_is_exported(lib):
    names = _lib.header_symbols()
    assert len(names) >= 18
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(_lib.SIGNATURES)


def test_struct_sizes_match_header_layout():
    assert C.sizeof(_lib.cmg_problem) == 20
    assert C.sizeof(_lib.cmg_stats) == 8 + 8 * 256
    assert C.sizeof(_lib.cmg_mem) == 8 * 8


def test_default_opts(lib):
    o = _lib.cmg_opts()
    assert lib.cmg_default_opts(C.byref(o)) == _lib.OK
    assert (o.smoother, o.nu_pre, o.nu_post, o.ir_iters, o.vcycles) == (_lib.RBGS, 2, 2, 2, 1)
    assert (o.bfp_block, o.bits_u, o.bits_r, o.bits_y, o.inc_u, o.inc_ry) == (64, 16, 16, 16, 2, 1)
    assert o.storage == _lib.COMPACT_BFP and o.vcycle_prec == _lib.FP32
    assert lib.cmg_default_opts(None) == _lib.INVALID_ARG


def _setup(lib, **kw):
    p = _lib.cmg_problem(3, 6, 1, _lib.POISSON, 1)
    o = _lib.cmg_opts()
    lib.cmg_default_opts(C.byref(o))
    for k, v in kw.items():
        if hasattr(p, k):
            setattr(p, k, v)
        else:
            setattr(o, k, v)
    ctx = C.c_void_p()
    st = lib.cmg_setup(C.byref(p), C.byref(o), None, None, C.byref(ctx))
    return st, ctx, lib.cmg_last_error(None).decode()


@pytest.mark.parametrize("kw,status", [
    (dict(dim=4), _lib.INVALID_ARG),
    (dict(L=1), _lib.INVALID_ARG),
    (dict(L=11), _lib.INVALID_ARG),
    (dict(coarsest=0), _lib.INVALID_ARG),
    (dict(coarsest=3), _lib.UNSUPPORTED),                  # dense coarsest solves hold at most 27 nodes
    (dict(coarsest=6), _lib.INVALID_ARG),                  # not below L
    (dict(keep_correction=2), _lib.INVALID_ARG),
    (dict(op=7), _lib.INVALID_ARG),
    (dict(op=_lib.DIFFUSION), _lib.INVALID_ARG),          # kappa missing
    (dict(batch=0), _lib.INVALID_ARG),
    (dict(vcycles=2), _lib.UNSUPPORTED),
    (dict(ir_iters=0), _lib.INVALID_ARG),
    (dict(bfp_block=48), _lib.INVALID_ARG),
    (dict(bits_u=1), _lib.INVALID_ARG),
    (dict(bits_u=54), _lib.INVALID_ARG),
    (dict(bits_r=25), _lib.INVALID_ARG),                   # > 24 with an FP32 V-cycle
    (dict(smoother=_lib.WJACOBI, omega=2.5), _lib.INVALID_ARG),
    (dict(nu_pre=-1), _lib.INVALID_ARG),
    (dict(storage=5), _lib.INVALID_ARG),
])
def test_setup_rejects_invalid(lib, kw, status):
    st, ctx, msg = _setup(lib, **kw)
    assert st == status
    assert not ctx.value
    assert msg


def test_null_arguments(lib):
    assert lib.cmg_setup(None, None, None, None, None) == _lib.INVALID_ARG
    assert lib.cmg_fmg_solve(None, None, None, None) == _lib.INVALID_ARG
    assert lib.cmg_vcycle(None, None, None) == _lib.INVALID_ARG
    assert lib.cmg_adjoint_solve(None, None, None, None, None) == _lib.INVALID_ARG
    assert lib.cmg_destroy(None) == _lib.INVALID_ARG
    assert lib.cmg_memory_stats(None, None) == _lib.INVALID_ARG
    assert isinstance(lib.cmg_last_error(None), bytes)


def test_noalloc_encode_rejects_sizes_beyond_its_workspace(lib):
    # checked before any HIP call: the static workspace holds 2^31 values
    assert lib.cmg_abfp_encode_noalloc(None, 1, (1 << 31) + 1, 16, None, None, None, None, None) == _lib.INVALID_ARG
    assert b"2^31" in lib.cmg_last_error(None)
    assert lib.cmg_abfp_encode_noalloc(None, 1, -1, 16, None, None, None, None, None) == _lib.INVALID_ARG


def test_code_bytes(lib):
    assert lib.cmg_bfp_code_bytes(100, 64, 8) == 128
    assert lib.cmg_bfp_code_bytes(100, 32, 12) == 128 * 12 // 8
    assert lib.cmg_bfp_code_bytes(64, 64, 16) == 128
    assert lib.cmg_bfp_code_bytes(1, 64, 17) == 256
    assert lib.cmg_bfp_code_bytes(10, 32, 53) == 256
    assert lib.cmg_bfp_code_bytes(10, 48, 8) == -1
    assert lib.cmg_bfp_code_bytes(10, 32, 1) == -1


def test_codec_rejects_bad_args_without_gpu(lib):
    assert lib.cmg_bfp_encode(None, 1, 10, 48, 8, None, None, None) == _lib.INVALID_ARG
    assert lib.cmg_bfp_encode(None, 1, 10, 64, 8, None, None, None) == _lib.INVALID_ARG
    assert lib.cmg_bfp_decode(None, None, 10, 64, 60, None, None) == _lib.INVALID_ARG
    assert lib.cmg_bfp_encode(None, 1, 0, 64, 8, None, None, None) == _lib.OK   # empty input
