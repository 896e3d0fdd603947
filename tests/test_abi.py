"""C-ABI conformance on the CPU: the library loads, exports every function the
public header declares, validates its arguments before touching a device, and
reports errors through status codes and stencil_last_error().  No compute call
is made here (there is no GPU in this tier)."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_2103_08825_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER_DIR = os.path.join(ROOT, "include")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2103_08825_amd import build
        build.build(incremental=True)
    return _lib.lib()


def _declared_functions():
    names = set()
    for fn in os.listdir(HEADER_DIR):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(HEADER_DIR, fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[a-z_][a-z_0-9 ]*\*?\s*\**\s*(stencil_[a-z_0-9]+)\s*\(",
                             text, flags=re.M):
            names.add(m.group(1))
    return names


def test_every_declared_symbol_is_exported(L):
    declared = _declared_functions()
    assert len(declared) >= 15, declared
    missing = [n for n in sorted(declared) if not hasattr(L, n)]
    assert not missing, missing
    assert set(_lib.EXPORTS) == declared


def test_version(L):
    assert _lib.stencil_version() == 1


@pytest.mark.parametrize("dim,r,kind", [(1, 1, 0), (1, 2, 1), (2, 1, 0), (2, 1, 1), (2, 2, 0), (3, 1, 0),
                                        (3, 1, 1), (3, 2, 0), (3, 4, 1), (2, 4, 0)])
def test_offsets_match_the_oracle_enumeration(L, dim, r, kind):
    got = np.array(_lib.stencil_offsets(dim, r, kind))
    ref = oracle.offsets(dim, r, kind)
    np.testing.assert_array_equal(got, ref)
    assert _lib.stencil_num_points(dim, r, kind) == len(ref)


def test_num_points_rejects_bad_arguments(L):
    for args in [(0, 1, 0), (4, 1, 0), (2, 0, 0), (2, 1, 2), (2, -1, 1)]:
        assert L.stencil_num_points(*args) == _lib.STENCIL_E_INVALID
        assert _lib.last_error() != ""


def _create(L, shape, r, kind, coeffs, bc, dtype, method=0, fused_k=0, variant=0, chunk=0):
    out = ctypes.c_void_p(123)
    sh = (ctypes.c_int64 * max(1, len(shape)))(*shape)
    c = (ctypes.c_double * max(1, len(coeffs)))(*coeffs)
    opts = _lib.Opts(method, fused_k, variant, 0, chunk)
    rc = L.stencil_plan_create(ctypes.byref(out), len(shape), sh, r, kind, c, len(coeffs), bc, dtype,
                               ctypes.byref(opts))
    return rc, out.value


@pytest.mark.parametrize("case,code", [
    (dict(shape=(8, 8), r=1, kind=0, coeffs=[0.2] * 4, bc=0, dtype=1), _lib.STENCIL_E_INVALID),
    (dict(shape=(8, 0), r=1, kind=0, coeffs=[0.2] * 5, bc=0, dtype=1), _lib.STENCIL_E_INVALID),
    (dict(shape=(8, 8), r=1, kind=0, coeffs=[0.2] * 5, bc=2, dtype=1), _lib.STENCIL_E_INVALID),
    (dict(shape=(8, 8), r=1, kind=0, coeffs=[0.2] * 5, bc=0, dtype=7), _lib.STENCIL_E_INVALID),
    (dict(shape=(8, 8), r=5, kind=0, coeffs=[0.0] * 21, bc=0, dtype=1), _lib.STENCIL_E_UNSUPPORTED),
    (dict(shape=(8, 8), r=1, kind=0, coeffs=[0.2] * 5, bc=0, dtype=1, method=9), _lib.STENCIL_E_INVALID),
    (dict(shape=(8, 8), r=1, kind=0, coeffs=[0.2] * 5, bc=0, dtype=1, method=2, fused_k=99),
     _lib.STENCIL_E_UNSUPPORTED),
    (dict(shape=(8, 8), r=1, kind=0, coeffs=[0.2] * 5, bc=0, dtype=1, method=2, variant=9),
     _lib.STENCIL_E_INVALID),
    (dict(shape=(8, 9), r=1, kind=0, coeffs=[0.2] * 5, bc=0, dtype=1, method=2, variant=2),
     _lib.STENCIL_E_INVALID),
    (dict(shape=(8, 8), r=1, kind=0, coeffs=[0.2] * 5, bc=0, dtype=1, chunk=-1), _lib.STENCIL_E_INVALID),
])
def test_plan_create_validation(L, case, code):
    rc, handle = _create(L, **case)
    assert rc == code
    assert handle is None                  # *out is NULL on failure
    assert _lib.last_error() != ""


def test_plan_create_allocates_nothing_and_resolves(L):
    rc, h = _create(L, (512, 512, 512), 1, 0, [1 / 7] * 7, 0, _lib.F32)
    assert rc == 0 and h
    info = _lib.stencil_plan_info(h)
    assert info["scratch_bytes"] == 0      # device memory only at the first run
    assert info["method"] == _lib.METHOD_FUSED and info["fused_k"] >= 1
    assert info["points"] == 512 ** 3 and info["elem_bytes"] == 4
    _lib.stencil_plan_destroy(h)
    # plain resolves to one step per launch, generic to the reference kernel
    for method, want in [(_lib.METHOD_PLAIN, _lib.METHOD_PLAIN), (_lib.METHOD_GENERIC, _lib.METHOD_GENERIC)]:
        rc, h = _create(L, (64, 64, 64), 1, 1, [1 / 27] * 27, 1, _lib.F64, method=method)
        info = _lib.stencil_plan_info(h)
        assert info["method"] == want and info["fused_k"] == 1
        _lib.stencil_plan_destroy(h)
    # a stencil without a compiled fused kernel falls back to the reference kernel under AUTO
    rc, h = _create(L, (16, 16, 16), 3, 1, [0.0] * 343, 0, _lib.F32)
    assert rc == 0 and _lib.stencil_plan_info(h)["method"] == _lib.METHOD_GENERIC
    _lib.stencil_plan_destroy(h)
    L.stencil_plan_destroy(None)           # NULL-safe


def test_run_and_adjoint_reject_bad_arguments_before_any_device_call(L):
    rc, h = _create(L, (32, 32), 1, 0, [0.2] * 5, 0, _lib.F32)
    assert L.stencil_run(h, None, ctypes.c_void_p(16), 3, None) == _lib.STENCIL_E_INVALID
    assert L.stencil_run(h, ctypes.c_void_p(16), ctypes.c_void_p(32), -1, None) == _lib.STENCIL_E_INVALID
    assert L.stencil_run(None, ctypes.c_void_p(16), ctypes.c_void_p(32), 1, None) == _lib.STENCIL_E_INVALID
    assert "NULL" in _lib.last_error() or "plan" in _lib.last_error()
    assert L.stencil_adjoint(h, ctypes.c_void_p(16), ctypes.c_void_p(32), 4, 0, ctypes.c_void_p(48),
                             ctypes.c_void_p(64), None) == _lib.STENCIL_E_INVALID
    rc, hb = _create(L, (32, 32), 1, 0, [0.2] * 5, 0, _lib.BF16)
    assert L.stencil_adjoint(hb, ctypes.c_void_p(16), ctypes.c_void_p(32), 4, 2, ctypes.c_void_p(48),
                             ctypes.c_void_p(64), None) == _lib.STENCIL_E_UNSUPPORTED
    assert L.stencil_reduce(9, ctypes.c_void_p(16), None, 4, ctypes.c_void_p(32), None) == _lib.STENCIL_E_INVALID
    assert L.stencil_reduce(1, ctypes.c_void_p(16), None, -1, ctypes.c_void_p(32), None) == _lib.STENCIL_E_INVALID
    _lib.stencil_plan_destroy(h)
    _lib.stencil_plan_destroy(hb)


def test_batched_rejects_bad_plans_before_any_device_call(L):
    rc, h3 = _create(L, (8, 8, 8), 1, 0, [1 / 7] * 7, 0, _lib.F32)
    rc, h2 = _create(L, (8, 8), 1, 0, [0.2] * 5, 0, _lib.F32)
    rc, hd = _create(L, (8, 8), 1, 0, [0.2] * 5, 0, _lib.F64)
    P = ctypes.c_void_p
    one = (ctypes.c_int64 * 2)(3, 3)
    out = P()

    def create(plans, ins, outs):
        n = len(plans)
        return L.stencil_batch_create(ctypes.byref(out), (P * n)(*plans), n, (P * n)(*ins), (P * n)(*outs),
                                      one, 0, None)
    assert create([h3], [16], [32]) == _lib.STENCIL_E_UNSUPPORTED
    assert create([h2], [16], [16]) == _lib.STENCIL_E_INVALID          # input aliases output
    assert create([h2, hd], [16, 48], [32, 64]) == _lib.STENCIL_E_INVALID  # mixed dtypes
    assert create([h2], [None], [32]) == _lib.STENCIL_E_INVALID
    assert out.value is None

    def create_flags(plans, ins, outs, flags):
        n = len(plans)
        return L.stencil_batch_create(ctypes.byref(out), (P * n)(*plans), n, (P * n)(*ins), (P * n)(*outs),
                                      one, flags, None)
    # unknown flag bits, and the item tuner (bit 1) rejects bad batches before it times anything
    assert create_flags([h2], [16], [32], 4) == _lib.STENCIL_E_INVALID
    assert create_flags([h2], [16], [16], 2) == _lib.STENCIL_E_INVALID
    assert create_flags([h3], [16], [32], 2) == _lib.STENCIL_E_UNSUPPORTED
    assert out.value is None
    assert L.stencil_batch_choice(None, None, None) == _lib.STENCIL_E_INVALID
    assert L.stencil_batch_launch(None, None) == _lib.STENCIL_E_INVALID
    assert L.stencil_batch_set_wait_limit(None, 10, None) == _lib.STENCIL_E_INVALID
    L.stencil_batch_destroy(None)
    for h in (h3, h2, hd):
        _lib.stencil_plan_destroy(h)


def test_error_text_is_thread_local(L):
    import threading
    L.stencil_num_points(0, 1, 0)
    main_msg = _lib.last_error()
    seen = []

    def worker():
        seen.append(_lib.last_error())
    t = threading.Thread(target=worker)
    t.start()
    t.join()
    assert main_msg != "" and seen == [""]


def test_requested_depth_picks_a_variant_compiled_that_deep(L):
    # the measured default tile of the 27-point FP32 box is compiled up to k = 3;
    # asking for k = 4 without a variant must choose a tile compiled that deep
    rc, h = _create(L, (64, 64, 64), 1, 1, [1 / 27] * 27, 0, _lib.F32, method=_lib.METHOD_FUSED, fused_k=4)
    assert rc == 0, _lib.last_error()
    info = _lib.stencil_plan_info(h)
    assert info["fused_k"] == 4 and info["variant"] != 0
    _lib.stencil_plan_destroy(h)
    rc, h = _create(L, (64, 64, 64), 1, 1, [1 / 27] * 27, 0, _lib.F32, method=_lib.METHOD_FUSED, fused_k=99)
    assert rc == _lib.STENCIL_E_UNSUPPORTED and "exceeds" in _lib.last_error()


def test_one_step_tile_follows_the_grid_size(L):
    # one-step sweeps keep the measured 512^3 tile on large grids and take the
    # smallest 3D tile, with chunks of at most 8 planes, below half of 512^3
    c7 = [0.1] * 7
    rc, h = _create(L, (512, 512, 512), 1, 0, c7, 0, _lib.F32, method=_lib.METHOD_PLAIN)
    assert rc == 0, _lib.last_error()
    big = _lib.stencil_plan_info(h)
    _lib.stencil_plan_destroy(h)
    rc, h = _create(L, (256, 256, 256), 1, 0, c7, 0, _lib.F32, method=_lib.METHOD_PLAIN)
    assert rc == 0, _lib.last_error()
    small = _lib.stencil_plan_info(h)
    _lib.stencil_plan_destroy(h)
    assert big["variant"] != 1 and small["variant"] == 1
    assert small["tile"][2] <= 8
    rc, h = _create(L, (128, 128, 128), 1, 0, c7, 0, _lib.F64, method=_lib.METHOD_PLAIN)
    assert rc == 0, _lib.last_error()
    f64 = _lib.stencil_plan_info(h)
    _lib.stencil_plan_destroy(h)
    assert f64["variant"] == 1 and f64["tile"][2] <= 8
    # the 27-point box and the 13-point star leave the one-step chunk to the
    # automatic rule, whose shortest chunk at k = 1 is 4(2r+1) planes
    for r, kind, n in ((1, 1, 27), (2, 0, 13)):
        rc, h = _create(L, (256, 256, 256), r, kind, [0.01] * n, 0, _lib.F32, method=_lib.METHOD_PLAIN)
        assert rc == 0, _lib.last_error()
        info = _lib.stencil_plan_info(h)
        _lib.stencil_plan_destroy(h)
        assert info["variant"] == 1 and info["tile"][2] == 4 * (2 * r + 1), (r, kind, info)


def test_tessellated_plans(L):
    # the tessellated method resolves on 3D grids with y extent >= 2(k+1)r and
    # reports its y tile; it refuses 2D grids, short y extents and depths
    # without a compiled kernel
    c7 = [0.1] * 7
    rc, h = _create(L, (512, 512, 512), 1, 0, c7, 0, _lib.F32, method=_lib.METHOD_TESSELLATE)
    assert rc == 0, _lib.last_error()
    info = _lib.stencil_plan_info(h)
    _lib.stencil_plan_destroy(h)
    assert info["method"] == _lib.METHOD_TESSELLATE and info["tile"][1] == 64
    rc, h = _create(L, (16, 11, 64), 1, 0, c7, 0, _lib.F32, method=_lib.METHOD_TESSELLATE, fused_k=5)
    assert rc == _lib.STENCIL_E_UNSUPPORTED and h is None
    assert "y extent" in _lib.last_error()
    rc, h = _create(L, (16, 12, 64), 1, 0, c7, 0, _lib.F32, method=_lib.METHOD_TESSELLATE, fused_k=5)
    assert rc == 0, _lib.last_error()
    _lib.stencil_plan_destroy(h)
    rc, h = _create(L, (64, 64), 1, 0, [0.2] * 5, 0, _lib.F32, method=_lib.METHOD_TESSELLATE)
    assert rc == _lib.STENCIL_E_UNSUPPORTED
    rc, h = _create(L, (16, 64, 64), 1, 0, c7, 0, _lib.F32, method=_lib.METHOD_TESSELLATE, fused_k=9)
    assert rc == _lib.STENCIL_E_UNSUPPORTED
