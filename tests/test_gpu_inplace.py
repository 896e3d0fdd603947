"""GPU parity of in-place fused passes (one field, no ping-pong copy; band
points of every output tile go through the side buffer): bit for bit against
the ping-pong plan with the same tile, depth and chunk, both when the output
is a second tensor and when it aliases the input, and against the FP64 oracle.
Shapes span several tiles and chunks with ragged tails, single tiles whose
periodic halo wraps onto themselves, and remainder passes."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import TOL, rel_err, rounded_inputs, say
from paper_2103_08825_amd import Plan
from paper_2103_08825_amd import workloads as W

pytestmark = pytest.mark.gpu

# (dim, r, kind, dtype, ks)
CASES = [(3, 1, W.STAR, "f32", (1, 3, 5)), (3, 1, W.BOX, "f32", (1, 3)), (3, 2, W.STAR, "f32", (2,)),
         (3, 1, W.STAR, "f64", (2, 3)), (3, 1, W.STAR, "bf16", (6,)), (3, 1, W.STAR, "f16", (4,)),
         (2, 1, W.STAR, "f32", (1, 5, 8)), (2, 1, W.BOX, "f32", (3, 8))]
SHAPES = {3: [(21, 70, 131), (9, 40, 30)], 2: [(45, 301), (40, 48)]}


@pytest.mark.parametrize("case", CASES, ids=lambda c: "%dd_r%d_%s_%s" % (c[0], c[1], "box" if c[2] else "star", c[3]))
@pytest.mark.parametrize("bc", [W.BC_ZERO, W.BC_PERIODIC])
def test_inplace_equals_pingpong_and_oracle(case, bc):
    dim, r, kind, dt, ks = case
    rng = np.random.default_rng(41)
    c = W.coefficients(rng, W.num_points(dim, r, kind))
    for shape in SHAPES[dim]:
        if dim == 2 and r == 1 and shape[1] % 4:
            continue
        u0 = rng.uniform(-1, 1, shape)
        t_in, u_ex, c_ex = rounded_inputs(u0, c, dt)
        x = t_in.cuda()
        for k in ks:
            ip = Plan(shape, r, kind, c, bc, dt, method="fused", fused_k=k, chunk=8, inplace=True)
            info = ip.info()
            pp = Plan(shape, r, kind, c, bc, dt, method="fused", fused_k=k, variant=info["variant"], chunk=8)
            for T in (k, 2 * k + 1):
                say("inplace %dD r=%d kind=%d %s bc=%d shape=%s k=%d variant=%d T=%d"
                    % (dim, r, kind, dt, bc, shape, k, info["variant"], T))
                ref = pp.run(x, T)
                got = ip.run(x, T)               # output in a second tensor
                z = x.clone()
                ip.run(z, T, out=z)              # output over the input
                torch.cuda.synchronize()
                assert torch.equal(got, ref), "in place (two tensors) != ping-pong"
                assert torch.equal(z, ref), "in place (aliased) != ping-pong"
            want = oracle.run(u_ex, c_ex, 2 * k + 1, r=r, kind=kind, bc=bc)
            assert rel_err(z.double().cpu().numpy(), want) <= TOL[dt]
            ip.close()
            pp.close()


def test_inplace_3d7p_512_footprint():
    """512^3 FP32 zero halo, T = 64, updated in place over its input, against
    the ping-pong plan; the in-place plan holds its side buffer only."""
    case = W.case_3d("3d7p", seed=0)
    x = torch.from_numpy(case.u0).float().cuda()
    pp = Plan(case.shape, 1, W.STAR, case.coeffs, W.BC_ZERO, "f32", method="fused")
    ref = pp.run(x, case.T)
    ip = Plan(case.shape, 1, W.STAR, case.coeffs, W.BC_ZERO, "f32", method="fused", inplace=True)
    z = x.clone()
    ip.run(z, case.T, out=z)
    torch.cuda.synchronize()
    assert torch.equal(z, ref)
    field = x.numel() * 4
    pi, ii = pp.info(), ip.info()
    say("512^3 FP32: ping-pong plan holds %.0f MiB, in-place plan %.0f MiB (field %.0f MiB)"
        % (pi["scratch_bytes"] / 2**20, ii["scratch_bytes"] / 2**20, field / 2**20))
    assert ii["scratch_bytes"] < field
