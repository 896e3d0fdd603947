"""Seeded synthetic inputs for stencil sweeps.

This module draws inputs only: coefficients, initial fields, targets and the
batched grid list.  It holds none of the stencil arithmetic and is the one
module that both the GPU path's callers and the CPU oracle's callers share.

The paper (Section 4.1, Table 1) runs synthetic grids of given shapes and
step counts and names no dataset; the distributions below are the readings
recorded in the design notes:
  * coefficients: w_j ~ U[0.5, 1.5) i.i.d., normalised c_j = w_j / sum(w) in FP64;
  * fields: U[-1, 1) i.i.d. in FP64 (cast by the caller to the storage dtype);
  * the 1D workload adds four zero-boundary sine modes 0.25*sin(pi*m*(i+1)/(N+1))
    with m drawn without replacement from [1, 1024];
  * adjoint targets: U[-1, 1);
  * draw order within one case: coefficients, field, sine modes, target.
Every case draws from numpy's PCG64 seeded with (seed, case tag).
"""
from __future__ import annotations

import dataclasses
import math
import zlib
from typing import List, Sequence, Tuple

import numpy as np

STAR, BOX = 0, 1
BC_ZERO, BC_PERIODIC = 0, 1


def num_points(dim: int, r: int, kind: int) -> int:
    return 2 * dim * r + 1 if kind == STAR else (2 * r + 1) ** dim


def rng_for(seed: int, tag: str) -> np.random.Generator:
    """PCG64 stream for one case, independent across tags."""
    return np.random.default_rng(np.random.SeedSequence([int(seed), zlib.crc32(tag.encode())]))


def coefficients(rng: np.random.Generator, npts: int) -> np.ndarray:
    w = rng.uniform(0.5, 1.5, size=npts)
    return w / w.sum()


def uniform_field(rng: np.random.Generator, shape: Sequence[int]) -> np.ndarray:
    return rng.uniform(-1.0, 1.0, size=tuple(int(s) for s in shape))


def sine_modes(rng: np.random.Generator, n: int, count: int = 4) -> np.ndarray:
    modes = rng.choice(np.arange(1, 1025), size=count, replace=False)
    i = np.arange(n, dtype=np.float64)
    out = np.zeros(n, dtype=np.float64)
    for m in modes:
        out += 0.25 * np.sin(math.pi * float(m) * (i + 1.0) / (n + 1.0))
    return out


@dataclasses.dataclass
class Case:
    """One stencil problem: shape (slowest axis first), order, kind, boundary, steps."""
    name: str
    shape: Tuple[int, ...]
    r: int
    kind: int
    bc: int
    T: int
    coeffs: np.ndarray
    u0: np.ndarray          # float64
    target: np.ndarray | None = None

    @property
    def dim(self) -> int:
        return len(self.shape)

    @property
    def npts(self) -> int:
        return num_points(self.dim, self.r, self.kind)


def make_case(name: str, shape, r: int, kind: int, bc: int, T: int, seed: int = 0,
              sines: bool = False, target: bool = False) -> Case:
    rng = rng_for(seed, name)
    shape = tuple(int(s) for s in shape)
    c = coefficients(rng, num_points(len(shape), r, kind))
    u0 = uniform_field(rng, shape)
    if sines:
        assert len(shape) == 1
        u0 = u0 + sine_modes(rng, shape[0])
    y = uniform_field(rng, shape) if target else None
    return Case(name, shape, r, kind, bc, T, c, u0, y)


# --- the paper-scale workloads -------------------------------------------------

def case_1d3p(seed: int = 0, n: int = 262_144, T: int = 200) -> Case:
    """1D 3-point star, zero halo, FP64 (plain one-step sweeps)."""
    return make_case("1d3p", (n,), 1, STAR, BC_ZERO, T, seed, sines=True)


def case_2d(kind: int, seed: int = 0, n: int = 8192, T: int = 100) -> Case:
    """2D 5-point star or 9-point box, periodic."""
    return make_case("2d5p" if kind == STAR else "2d9p", (n, n), 1, kind, BC_PERIODIC, T, seed)


def case_3d(name: str, seed: int = 0, n: int = 512, T: int = 64) -> Case:
    """3D 7-point star (r=1), 13-point star (r=2) or 27-point box (r=1), zero halo."""
    r, kind = {"3d7p": (1, STAR), "3d13p": (2, STAR), "3d27p": (1, BOX)}[name]
    return make_case(name, (n, n, n), r, kind, BC_ZERO, T, seed)


def case_adjoint(seed: int = 0, n: int = 256, T: int = 100) -> Case:
    """3D 7-point star, periodic, with a random target for L = 0.5*||u_T - y||^2."""
    return make_case("adj3d7p", (n, n, n), 1, STAR, BC_PERIODIC, T, seed, target=True)


# The six problems of the paper's evaluation (Section 4.1, Table 1): FP64, T = 1000.
# The paper does not state a boundary rule; the zero halo is used.
TABLE1 = (("t1_1d3p", (10_240_000,), 1, STAR), ("t1_1d5p", (10_240_000,), 2, STAR),
          ("t1_2d5p", (3000, 3000), 1, STAR), ("t1_2d9p", (3000, 3000), 1, BOX),
          ("t1_3d7p", (128, 128, 128), 1, STAR), ("t1_3d27p", (128, 128, 128), 1, BOX))


def case_table1(name: str, seed: int = 0, T: int = 1000) -> Case:
    """One of the Table 1 problems by name (t1_1d3p ... t1_3d27p), zero halo."""
    for n, shape, r, kind in TABLE1:
        if n == name:
            return make_case(n, shape, r, kind, BC_ZERO, T, seed)
    raise KeyError(name)


@dataclasses.dataclass
class BatchedGrid:
    shape: Tuple[int, int]
    kind: int
    T: int
    coeffs: np.ndarray
    seed_tag: str


def batched_grids(seed: int = 0, count: int = 256, lo: int = 64, hi: int = 2048,
                  tmin: int = 10, tmax: int = 200) -> List[BatchedGrid]:
    """Independent 2D grids: sides log-uniform in [lo, hi] per axis, each a 5-point
    star or a 9-point box with probability 1/2, T uniform in [tmin, tmax]."""
    rng = rng_for(seed, "batched")
    out = []
    for i in range(count):
        sy = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        sx = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        kind = STAR if rng.uniform() < 0.5 else BOX
        T = int(rng.integers(tmin, tmax + 1))
        c = coefficients(rng, num_points(2, 1, kind))
        out.append(BatchedGrid((sy, sx), kind, T, c, "batched/%d" % i))
    return out


def batched_field(seed: int, grid: BatchedGrid) -> np.ndarray:
    return uniform_field(rng_for(seed, grid.seed_tag), grid.shape)


# --- exact (dyadic) inputs ----------------------------------------------------

def dyadic_coefficients(dim: int, r: int, kind: int) -> np.ndarray:
    """Power-of-two weights summing exactly to 1: the centre takes 1/2 and the
    other npts-1 points share 1/2 in equal power-of-two parts where possible,
    otherwise a power-of-two split of the remainder."""
    n = num_points(dim, r, kind)
    others = n - 1
    # largest power of two p with p >= others; give each non-centre point 1/(2p)
    p = 1
    while p < others:
        p *= 2
    w = np.full(n, 1.0 / (2 * p))
    centre = n // 2
    w[centre] = 1.0 - (others / (2.0 * p))
    return w


def dyadic_field(rng: np.random.Generator, shape, lo: int = -8, hi: int = 8) -> np.ndarray:
    return rng.integers(lo, hi + 1, size=tuple(shape)).astype(np.float64)
