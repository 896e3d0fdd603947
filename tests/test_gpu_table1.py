"""GPU parity on the six problems of the paper's evaluation (Section 4.1, Table 1):
1D 3- and 5-point stars on 10,240,000 points, 2D 5-point star and 9-point box
on 3000^2, 3D 7-point star and 27-point box on 128^3, FP64, T = 1000, zero
halo, in the library's default launch configuration.

The 3D results are compared with the FP64 oracle on the whole field; the 1D and
2D results on sampled blocks (grid ends and interior in 1D, opposite corners in
2D), each computed by the oracle from its own dependency cone (the block widened
by T*r on every side).  Tolerance 1e-12 normwise (FP64).
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import rel_err, say
from paper_2103_08825_amd import Plan
from paper_2103_08825_amd import workloads as W

pytestmark = pytest.mark.gpu

# Sample blocks; in 2D the two opposite corners keep the oracle's dependency
# cones (about 1000^2 points each) affordable, and each cone spans hundreds of
# the kernel's interior tiles, so an error anywhere in it reaches the block.
BLOCKS = {
    1: [(0,), (5_120_000,), (10_240_000 - 4,)],
    2: [(0, 0), (2996, 2996)],
}


@pytest.mark.parametrize("name", [t[0] for t in W.TABLE1])
def test_table1_fp64(name):
    case = W.case_table1(name)
    plan = Plan(case.shape, case.r, case.kind, case.coeffs, case.bc, "f64")
    info = plan.info()
    say("%s %s T=%d plan k=%d variant=%d tile=%s" % (name, case.shape, case.T, info["fused_k"], info["variant"],
                                                      info["tile"]))
    got = plan.run(torch.from_numpy(case.u0).cuda(), case.T).cpu().numpy()
    if case.dim == 3:
        ref = oracle.run(case.u0, case.coeffs, case.T, r=case.r, kind=case.kind, bc=case.bc)
        err = rel_err(got, ref)
        say("  whole field: rel err %.3e (max|ref| %.3e)" % (err, np.abs(ref).max()))
        assert err <= 1e-12
        return
    size = (4,) * case.dim
    gs, rs = [], []
    for start in BLOCKS[case.dim]:
        sz = tuple(min(b, n - s) for b, n, s in zip(size, case.shape, start))
        ref = oracle.block_run(case.u0, case.coeffs, case.T, start, sz, r=case.r, kind=case.kind, bc=case.bc)
        sl = tuple(slice(s, s + b) for s, b in zip(start, sz))
        gs.append(got[sl].ravel())
        rs.append(ref.ravel())
    g, r = np.concatenate(gs), np.concatenate(rs)
    err = rel_err(g, r)
    say("  %d sampled blocks: rel err %.3e (max|ref| %.3e)" % (len(gs), err, np.abs(r).max()))
    assert err <= 1e-12
    # the whole field: max-norm contraction (positive weights summing to 1)
    assert np.abs(got).max() <= np.abs(case.u0).max() * (1 + 1e-12)
