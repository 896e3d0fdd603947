"""The allocation-free reduction (stencil_reduce_noalloc) against the
allocating one (stencil_reduce), called through the C ABI: two calls in a row
per storage type, the second on a smaller input, each bitwise equal to
stencil_reduce on the same data (the same kernels and partial layout) and
within FP64 rounding of a NumPy reference."""
import numpy as np
import pytest
import torch

from gpu_util import TORCH, say
from paper_2103_08825_amd import _lib

pytestmark = pytest.mark.gpu

CODE = {"f64": _lib.F64, "f32": _lib.F32, "bf16": _lib.BF16, "f16": _lib.F16}


def _reduce(fn, dt, a, b):
    out = torch.full((6,), float("nan"), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    fn(CODE[dt], a.data_ptr(), b.data_ptr() if b is not None else 0, a.numel(), out.data_ptr(), stream)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("dt", ["f64", "f32", "bf16", "f16"])
def test_noalloc_reduce_matches_allocating_reduce(dt):
    rng = np.random.default_rng(21)
    for n in ((3 << 20) + 5, 1001):   # the second call is smaller than the first
        a = torch.from_numpy(rng.uniform(-1, 1, n)).to(TORCH[dt]).cuda()
        b = torch.from_numpy(rng.uniform(-1, 1, n)).to(TORCH[dt]).cuda()
        for ref_arg in (b, None):
            say("noalloc reduce %s n=%d ref=%s" % (dt, n, ref_arg is not None))
            want = _reduce(_lib.stencil_reduce, dt, a, ref_arg)
            got = _reduce(_lib.stencil_reduce_noalloc, dt, a, ref_arg)
            np.testing.assert_array_equal(got, want)
            x = a.double().cpu().numpy()
            ref = [x.sum(), (x * x).sum(), np.abs(x).max()]
            if ref_arg is not None:
                y = b.double().cpu().numpy()
                ref += [((x - y) ** 2).sum(), np.abs(x - y).max(), np.abs(y).max()]
            else:
                ref += [0.0, 0.0, 0.0]
            np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-9)


def test_noalloc_reduce_argument_errors():
    L = _lib.lib()
    import ctypes
    assert L.stencil_reduce_noalloc(9, ctypes.c_void_p(16), None, 4, ctypes.c_void_p(32), None) == _lib.STENCIL_E_INVALID
    assert L.stencil_reduce_noalloc(1, ctypes.c_void_p(16), None, -1, ctypes.c_void_p(32), None) == _lib.STENCIL_E_INVALID
    assert L.stencil_reduce_noalloc(1, None, None, 4, ctypes.c_void_p(32), None) == _lib.STENCIL_E_INVALID
    # n = 0: all six results are 0
    out = torch.full((6,), 7.0, dtype=torch.float64, device="cuda")
    dummy = torch.zeros(1, device="cuda")
    _lib.stencil_reduce_noalloc(_lib.F32, dummy.data_ptr(), 0, 0, out.data_ptr(),
                                torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert (out.cpu().numpy() == 0).all()
