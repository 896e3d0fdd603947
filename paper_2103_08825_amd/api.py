"""Torch-facing wrappers over the C ABI: plans, sweeps, reductions.

Tensors supply device memory and torch's current HIP stream supplies the
stream; every step of a sweep runs in the library's HIP kernels.
"""
from __future__ import annotations

from typing import Sequence

import torch

from . import _lib
from ._lib import (BC_PERIODIC, BC_ZERO, BOX, F16, F32, F64, BF16, METHOD_AUTO, METHOD_FUSED,
                   METHOD_GENERIC, METHOD_PLAIN, METHOD_TESSELLATE, STAR)

TORCH_DTYPE = {F64: torch.float64, F32: torch.float32, BF16: torch.bfloat16, F16: torch.float16}
CODE_OF = {v: k for k, v in TORCH_DTYPE.items()}
METHODS = {"auto": METHOD_AUTO, "plain": METHOD_PLAIN, "fused": METHOD_FUSED,
           "generic": METHOD_GENERIC, "tessellate": METHOD_TESSELLATE}


def dtype_code(dtype) -> int:
    if isinstance(dtype, int):
        return dtype
    if isinstance(dtype, str):
        return {"f64": F64, "f32": F32, "bf16": BF16, "f16": F16}[dtype]
    return CODE_OF[dtype]


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _check_tensor(t: torch.Tensor, dtype: torch.dtype, numel: int, name: str):
    if not t.is_cuda:
        raise ValueError("%s must be a GPU tensor" % name)
    if t.dtype != dtype:
        raise ValueError("%s has dtype %s, the plan needs %s" % (name, t.dtype, dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.numel() != numel:
        raise ValueError("%s has %d elements, the plan needs %d" % (name, t.numel(), numel))


class Plan:
    """A d-dimensional star or box stencil of order r on a fixed grid shape.

    coeffs are in canonical order (``offsets(dim, r, kind)``).  With graph=True,
    run() records its launches for an (input, output, T) triple into a HIP graph
    on the first call and replays it while later calls repeat the triple.  With
    inplace=True the passes update the output field in place (no ping-pong field;
    run(x, T, out=x) needs no copy of x)."""

    def __init__(self, shape: Sequence[int], r: int, kind: int, coeffs, bc: int, dtype,
                 method: str | int = "auto", fused_k: int = 0, variant: int = 0,
                 autotune: bool = False, chunk: int = 0, graph: bool = False,
                 inplace: bool = False):
        self.shape = tuple(int(s) for s in shape)
        self.r, self.kind, self.bc = int(r), int(kind), int(bc)
        self.dtype_code = dtype_code(dtype)
        self.dtype = TORCH_DTYPE[self.dtype_code]
        self.coeffs = [float(c) for c in coeffs]
        m = METHODS[method] if isinstance(method, str) else int(method)
        self.handle = _lib.stencil_plan_create(self.shape, self.r, self.kind, self.coeffs, self.bc,
                                               self.dtype_code, m, int(fused_k), int(variant),
                                               autotune, int(chunk), bool(graph), bool(inplace))
        self.numel = 1
        for s in self.shape:
            self.numel *= s

    @property
    def dim(self) -> int:
        return len(self.shape)

    def info(self) -> dict:
        return _lib.stencil_plan_info(self.handle)

    def prepare(self) -> None:
        _lib.stencil_plan_prepare(self.handle, _stream())

    def autotune(self) -> dict:
        _lib.stencil_autotune(self.handle, _stream())
        return self.info()

    def run(self, u0: torch.Tensor, T: int, out: torch.Tensor | None = None) -> torch.Tensor:
        """u_T after T steps; enqueued on torch's current stream."""
        _check_tensor(u0, self.dtype, self.numel, "u0")
        if out is None:
            out = torch.empty(self.shape, dtype=self.dtype, device=u0.device)
        _check_tensor(out, self.dtype, self.numel, "out")
        _lib.stencil_run(self.handle, u0.data_ptr(), out.data_ptr(), int(T), _stream())
        return out

    def adjoint(self, u0: torch.Tensor, gT: torch.Tensor, T: int, ckpt: int = 10):
        """(dL/du0, dL/dc) of u_T = run(u0, T) for dL/du_T = gT.  dL/dc is FP64, one
        entry per coefficient in canonical order."""
        _check_tensor(u0, self.dtype, self.numel, "u0")
        _check_tensor(gT, self.dtype, self.numel, "gT")
        grad_u0 = torch.empty(self.shape, dtype=self.dtype, device=u0.device)
        grad_c = torch.empty(len(self.coeffs), dtype=torch.float64, device=u0.device)
        _lib.stencil_adjoint(self.handle, u0.data_ptr(), gT.data_ptr(), int(T), int(ckpt),
                             grad_u0.data_ptr(), grad_c.data_ptr(), _stream())
        return grad_u0, grad_c

    def close(self) -> None:
        if getattr(self, "handle", None):
            _lib.stencil_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def offsets(dim: int, r: int, kind: int):
    return _lib.stencil_offsets(dim, r, kind)


def num_points(dim: int, r: int, kind: int) -> int:
    return _lib.stencil_num_points(dim, r, kind)


def reduce(u: torch.Tensor, ref: torch.Tensor | None = None) -> torch.Tensor:
    """FP64 [sum u, sum u^2, max|u|, sum (u-ref)^2, max|u-ref|, max|ref|] (device tensor)."""
    code = CODE_OF[u.dtype]
    if not u.is_cuda or not u.is_contiguous():
        raise ValueError("u must be a contiguous GPU tensor")
    if ref is not None:
        _check_tensor(ref, u.dtype, u.numel(), "ref")
    out = torch.empty(6, dtype=torch.float64, device=u.device)
    _lib.stencil_reduce(code, u.data_ptr(), ref.data_ptr() if ref is not None else 0, u.numel(),
                        out.data_ptr(), _stream())
    return out
