"""ctypes marshalling for libstencil.so: one Python function per C entry point.

Every function takes plain Python ints (device pointers, stream handles) and
sequences; no computation happens here.  The library must have been built
(``python -m paper_2103_08825_amd.build``): loading fails loudly otherwise,
and there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libstencil.so")

STENCIL_OK = 0
STENCIL_E_INVALID = -1
STENCIL_E_UNSUPPORTED = -2
STENCIL_E_NOMEM = -3
STENCIL_E_DEVICE = -4
STAR, BOX = 0, 1
BC_ZERO, BC_PERIODIC = 0, 1
F64, F32, BF16, F16 = 0, 1, 2, 3
METHOD_AUTO, METHOD_PLAIN, METHOD_FUSED, METHOD_GENERIC, METHOD_TESSELLATE = 0, 1, 2, 3, 4
MAX_DIM = 3

# Every symbol include/stencil.h declares.
EXPORTS = (
    "stencil_num_points", "stencil_offsets", "stencil_plan_create", "stencil_plan_destroy",
    "stencil_plan_info", "stencil_plan_prepare", "stencil_autotune", "stencil_run",
    "stencil_run_batched", "stencil_batch_create", "stencil_batch_launch", "stencil_batch_destroy",
    "stencil_batch_info", "stencil_batch_choice", "stencil_batch_status", "stencil_batch_set_wait_limit", "stencil_adjoint", "stencil_reduce", "stencil_reduce_noalloc", "stencil_last_error",
    "stencil_version",
)


class StencilError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__("%s failed (%d): %s" % (where, code, msg))
        self.code = code


class Opts(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int), ("fused_k", ctypes.c_int), ("variant", ctypes.c_int),
                ("autotune", ctypes.c_int), ("chunk", ctypes.c_int), ("graph", ctypes.c_int),
                ("inplace", ctypes.c_int)]


class PlanDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("radius", ctypes.c_int), ("kind", ctypes.c_int),
                ("bc", ctypes.c_int), ("dtype", ctypes.c_int), ("npts", ctypes.c_int),
                ("shape", ctypes.c_int64 * MAX_DIM), ("points", ctypes.c_int64),
                ("method", ctypes.c_int), ("fused_k", ctypes.c_int), ("variant", ctypes.c_int),
                ("tile", ctypes.c_int * 3), ("elem_bytes", ctypes.c_int),
                ("scratch_bytes", ctypes.c_int64), ("tuned", ctypes.c_int)]


_lock = threading.Lock()
_lib = None


def lib():
    """Load libstencil.so (once) and declare the C signatures."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libstencil.so is not built (%s); run "
                               "`python -m paper_2103_08825_amd.build`" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32, ci, cd = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int, ctypes.c_double
        P = ctypes.POINTER
        sig = {
            "stencil_num_points": (ci, [ci, ci, ci]),
            "stencil_offsets": (ci, [ci, ci, ci, P(i32)]),
            "stencil_plan_create": (ci, [P(vp), ci, P(i64), ci, ci, P(cd), ci, ci, ci, P(Opts)]),
            "stencil_plan_destroy": (None, [vp]),
            "stencil_plan_info": (ci, [vp, P(PlanDesc)]),
            "stencil_plan_prepare": (ci, [vp, vp]),
            "stencil_autotune": (ci, [vp, vp]),
            "stencil_run": (ci, [vp, vp, vp, i64, vp]),
            "stencil_run_batched": (ci, [P(vp), ci, P(vp), P(vp), P(i64), vp]),
            "stencil_batch_create": (ci, [P(vp), P(vp), ci, P(vp), P(vp), P(i64), ci, vp]),
            "stencil_batch_launch": (ci, [vp, vp]),
            "stencil_batch_destroy": (None, [vp]),
            "stencil_batch_info": (ci, [vp, P(i64), P(i64)]),
            "stencil_batch_choice": (ci, [vp, P(ci), P(ci)]),
            "stencil_batch_status": (ci, [vp, vp]),
            "stencil_batch_set_wait_limit": (ci, [vp, i64, vp]),
            "stencil_adjoint": (ci, [vp, vp, vp, i64, i64, vp, vp, vp]),
            "stencil_reduce": (ci, [ci, vp, vp, i64, vp, vp]),
            "stencil_reduce_noalloc": (ci, [ci, vp, vp, i64, vp, vp]),
            "stencil_last_error": (ctypes.c_char_p, []),
            "stencil_version": (ci, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
        return L


def last_error() -> str:
    return lib().stencil_last_error().decode(errors="replace")


def check(rc: int, where: str) -> int:
    if rc < 0:
        raise StencilError(rc, where, last_error())
    return rc


def _ptrs(seq):
    arr = (ctypes.c_void_p * len(seq))()
    for i, v in enumerate(seq):
        arr[i] = int(v) if v else None
    return arr


# --- one wrapper per entry point ---------------------------------------------

def stencil_num_points(dim: int, radius: int, kind: int) -> int:
    return check(lib().stencil_num_points(dim, radius, kind), "stencil_num_points")


def stencil_offsets(dim: int, radius: int, kind: int):
    n = stencil_num_points(dim, radius, kind)
    buf = (ctypes.c_int32 * (n * dim))()
    check(lib().stencil_offsets(dim, radius, kind, buf), "stencil_offsets")
    return [tuple(buf[j * dim:(j + 1) * dim]) for j in range(n)]


def stencil_plan_create(shape, radius: int, kind: int, coeffs, bc: int, dtype: int,
                        method: int = METHOD_AUTO, fused_k: int = 0, variant: int = 0,
                        autotune: bool = False, chunk: int = 0, graph: bool = False,
                        inplace: bool = False) -> int:
    dim = len(shape)
    sh = (ctypes.c_int64 * max(dim, 1))(*[int(s) for s in shape])
    c = (ctypes.c_double * len(coeffs))(*[float(v) for v in coeffs])
    opts = Opts(method, fused_k, variant, 1 if autotune else 0, chunk, 1 if graph else 0,
                1 if inplace else 0)
    out = ctypes.c_void_p()
    check(lib().stencil_plan_create(ctypes.byref(out), dim, sh, radius, kind, c, len(coeffs), bc,
                                    dtype, ctypes.byref(opts)), "stencil_plan_create")
    return out.value


def stencil_plan_destroy(plan: int) -> None:
    lib().stencil_plan_destroy(plan)


def stencil_plan_info(plan: int) -> dict:
    d = PlanDesc()
    check(lib().stencil_plan_info(plan, ctypes.byref(d)), "stencil_plan_info")
    return {"dim": d.dim, "radius": d.radius, "kind": d.kind, "bc": d.bc, "dtype": d.dtype,
            "npts": d.npts, "shape": tuple(d.shape[:d.dim]), "points": d.points,
            "method": d.method, "fused_k": d.fused_k, "variant": d.variant,
            "tile": tuple(d.tile), "elem_bytes": d.elem_bytes, "scratch_bytes": d.scratch_bytes,
            "tuned": d.tuned}


def stencil_plan_prepare(plan: int, stream: int) -> None:
    check(lib().stencil_plan_prepare(plan, stream), "stencil_plan_prepare")


def stencil_autotune(plan: int, stream: int) -> None:
    check(lib().stencil_autotune(plan, stream), "stencil_autotune")


def stencil_run(plan: int, d_in: int, d_out: int, T: int, stream: int) -> None:
    check(lib().stencil_run(plan, d_in, d_out, int(T), stream), "stencil_run")


def stencil_run_batched(plans, d_in, d_out, Ts, stream: int) -> None:
    n = len(plans)
    check(lib().stencil_run_batched(_ptrs(plans), n, _ptrs(d_in), _ptrs(d_out),
                                    (ctypes.c_int64 * n)(*[int(t) for t in Ts]), stream),
          "stencil_run_batched")


def stencil_batch_create(plans, d_in, d_out, Ts, flags: int, stream: int) -> int:
    n = len(plans)
    out = ctypes.c_void_p()
    check(lib().stencil_batch_create(ctypes.byref(out), _ptrs(plans), n, _ptrs(d_in), _ptrs(d_out),
                                     (ctypes.c_int64 * n)(*[int(t) for t in Ts]), flags, stream),
          "stencil_batch_create")
    return out.value


def stencil_batch_launch(batch: int, stream: int) -> None:
    check(lib().stencil_batch_launch(batch, stream), "stencil_batch_launch")


def stencil_batch_destroy(batch: int) -> None:
    lib().stencil_batch_destroy(batch)


def stencil_batch_info(batch: int):
    items, wgs = ctypes.c_int64(), ctypes.c_int64()
    check(lib().stencil_batch_info(batch, ctypes.byref(items), ctypes.byref(wgs)), "stencil_batch_info")
    return items.value, wgs.value


def stencil_batch_choice(batch: int):
    """(depths for order-1 star, order-1 box, order-2 star, order-2 box; rows per item)"""
    depths, chunk = (ctypes.c_int * 4)(), ctypes.c_int()
    check(lib().stencil_batch_choice(batch, depths, ctypes.byref(chunk)), "stencil_batch_choice")
    return list(depths), chunk.value


def stencil_batch_status(batch: int, stream: int) -> None:
    check(lib().stencil_batch_status(batch, stream), "stencil_batch_status")


def stencil_batch_set_wait_limit(batch: int, limit_us: int, stream: int) -> None:
    check(lib().stencil_batch_set_wait_limit(batch, int(limit_us), stream), "stencil_batch_set_wait_limit")


def stencil_adjoint(plan: int, d_u0: int, d_gT: int, T: int, ckpt: int, d_grad_u0: int,
                    d_grad_c: int, stream: int) -> None:
    check(lib().stencil_adjoint(plan, d_u0, d_gT, int(T), int(ckpt), d_grad_u0, d_grad_c, stream),
          "stencil_adjoint")


def stencil_reduce(dtype: int, d_u: int, d_ref: int, n: int, d_out: int, stream: int) -> None:
    check(lib().stencil_reduce(dtype, d_u, d_ref or None, int(n), d_out, stream), "stencil_reduce")


def stencil_reduce_noalloc(dtype: int, d_u: int, d_ref: int, n: int, d_out: int, stream: int) -> None:
    check(lib().stencil_reduce_noalloc(dtype, d_u, d_ref or None, int(n), d_out, stream),
          "stencil_reduce_noalloc")


def stencil_version() -> int:
    return lib().stencil_version()
