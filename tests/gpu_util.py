"""Helpers shared by the GPU parity tests: dtype rounding of the inputs the GPU
receives, the normwise error metric, and a small runner around Plan."""
from __future__ import annotations

import sys

import numpy as np
import torch

TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 2e-2, "f16": 2e-2}
TORCH = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rounded_inputs(u0: np.ndarray, coeffs: np.ndarray, dt: str):
    """The exact values the GPU receives, as FP64: the field rounded to the
    storage type and, below FP64, the weights rounded to FP32."""
    t = torch.from_numpy(np.ascontiguousarray(u0, dtype=np.float64)).to(TORCH[dt])
    u_exact = t.to(torch.float64).numpy()
    c = np.asarray(coeffs, dtype=np.float64)
    c_exact = c if dt == "f64" else c.astype(np.float32).astype(np.float64)
    return t, u_exact, c_exact


def rel_err(got: np.ndarray, ref: np.ndarray) -> float:
    """max |got - ref| / max |ref| (absolute error when ref is all zero)."""
    den = float(np.max(np.abs(ref))) if ref.size else 0.0
    num = float(np.max(np.abs(np.asarray(got, dtype=np.float64) - ref))) if ref.size else 0.0
    return num / den if den > 1e-300 else num


def gpu_sweep(plan, t_in: torch.Tensor, T: int) -> np.ndarray:
    d_in = t_in.to("cuda")
    out = plan.run(d_in, T)
    torch.cuda.synchronize()
    return out.to(torch.float64).cpu().numpy()


def record_error(key: str, rec: dict) -> None:
    """Adds one result's error record to the JSON file named by the environment
    variable STENCIL_ERROR_TABLE (no-op when it is unset)."""
    import json
    import os
    path = os.environ.get("STENCIL_ERROR_TABLE")
    if not path:
        return
    table = {}
    if os.path.exists(path):
        with open(path) as f:
            table = json.load(f)
    table[key] = rec
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
