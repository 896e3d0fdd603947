"""Batched sweeps: many independent 2D grids in one persistent, graph-captured launch."""
from __future__ import annotations

from typing import Sequence

import torch

from . import _lib
from .api import Plan, _check_tensor, _stream


class Batch:
    """A captured batched sweep.  Plans and tensors must outlive it."""

    def __init__(self, plans: Sequence[Plan], inputs: Sequence[torch.Tensor],
                 outputs: Sequence[torch.Tensor], Ts: Sequence[int], autotune: bool = False,
                 tune_items: bool = False):
        """autotune: tune each plan on single-grid launches and take its depth;
        tune_items: tune the items' depth and rows on this batch's persistent
        kernel (creation replays the batch several times, overwriting outputs)."""
        if not (len(plans) == len(inputs) == len(outputs) == len(Ts)):
            raise ValueError("plans, inputs, outputs and Ts differ in length")
        for p, x, y in zip(plans, inputs, outputs):
            _check_tensor(x, p.dtype, p.numel, "input")
            _check_tensor(y, p.dtype, p.numel, "output")
        self._keep = (list(plans), list(inputs), list(outputs))
        self.handle = _lib.stencil_batch_create([p.handle for p in plans],
                                                [x.data_ptr() for x in inputs],
                                                [y.data_ptr() for y in outputs], list(Ts),
                                                (1 if autotune else 0) | (2 if tune_items else 0),
                                                _stream())

    def launch(self) -> None:
        _lib.stencil_batch_launch(self.handle, _stream())

    def status(self) -> None:
        _lib.stencil_batch_status(self.handle, _stream())

    def set_wait_limit(self, limit_us: int) -> None:
        """How long an item polls for its grid's previous pass before giving up
        (microseconds; default one second)."""
        _lib.stencil_batch_set_wait_limit(self.handle, limit_us, _stream())

    def info(self):
        return _lib.stencil_batch_info(self.handle)

    def choice(self):
        """([order-1 star, order-1 box, order-2 star, order-2 box] depths, rows per item)"""
        return _lib.stencil_batch_choice(self.handle)

    def close(self) -> None:
        if getattr(self, "handle", None):
            _lib.stencil_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_batched(plans: Sequence[Plan], inputs: Sequence[torch.Tensor],
                outputs: Sequence[torch.Tensor], Ts: Sequence[int]) -> None:
    for p, x, y in zip(plans, inputs, outputs):
        _check_tensor(x, p.dtype, p.numel, "input")
        _check_tensor(y, p.dtype, p.numel, "output")
    _lib.stencil_run_batched([p.handle for p in plans], [x.data_ptr() for x in inputs],
                             [y.data_ptr() for y in outputs], list(Ts), _stream())
