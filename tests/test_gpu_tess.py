"""GPU parity of the tessellated fused sweep (Section 3.4 tiling along y):
bit for bit against the overlapped fused sweep with the same tile and depth
(every intermediate level is computed by the same arithmetic and kept in
compute precision), and against the FP64 oracle within the dtype's
tolerance.  Shapes cover several y tiles, a short last tile merged with the
one before it, a single tile, ragged x and z tails, both boundary rules and
remainder passes (T mod k != 0)."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import TOL, TORCH, rel_err, rounded_inputs, say
from paper_2103_08825_amd import Plan
from paper_2103_08825_amd import workloads as W

pytestmark = pytest.mark.gpu

# (name, r, kind, dtype, ks)
CASES = [("3d7p", 1, W.STAR, "f32", (1, 3, 5, 6)), ("3d27p", 1, W.BOX, "f32", (1, 2, 3)),
         ("3d13p", 2, W.STAR, "f32", (1, 2)), ("3d7p", 1, W.STAR, "bf16", (2, 6)),
         ("3d7p", 1, W.STAR, "f16", (3,)), ("3d7p", 1, W.STAR, "f64", (1, 3))]
SHAPES = [(20, 133, 150), (13, 100, 70), (9, 64, 131), (11, 40, 64)]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "%s_%s" % (c[0], c[3]))
@pytest.mark.parametrize("bc", [W.BC_ZERO, W.BC_PERIODIC])
def test_tessellated_equals_fused_and_oracle(case, bc):
    name, r, kind, dt, ks = case
    rng = np.random.default_rng(31)
    c = W.coefficients(rng, W.num_points(3, r, kind))
    for shape in SHAPES:
        u0 = rng.uniform(-1, 1, shape)
        t_in, u_ex, c_ex = rounded_inputs(u0, c, dt)
        x = t_in.cuda()
        for k in ks:
            if shape[1] < 2 * (k + 1) * r:
                continue
            tess = Plan(shape, r, kind, c, bc, dt, method="tessellate", fused_k=k, chunk=8)
            info = tess.info()
            fused = Plan(shape, r, kind, c, bc, dt, method="fused", fused_k=k, variant=info["variant"], chunk=8)
            for T in (k, 2 * k + 1):
                say("tess %s %s bc=%d shape=%s k=%d variant=%d T=%d" % (name, dt, bc, shape, k, info["variant"], T))
                got = tess.run(x, T)
                ref = fused.run(x, T)
                torch.cuda.synchronize()
                assert torch.equal(got, ref), "tessellated != fused"
            want = oracle.run(u_ex, c_ex, 2 * k + 1, r=r, kind=kind, bc=bc)
            err = rel_err(got.double().cpu().numpy(), want)
            assert err <= TOL[dt], err
            tess.close()
            fused.close()


def test_tessellated_3d7p_512_equals_fused():
    """The headline grid: 512^3 FP32 zero halo, T = 64, at the fused method's
    default depth and tile."""
    case = W.case_3d("3d7p", seed=0)
    x = torch.from_numpy(case.u0).float().cuda()
    tess = Plan(case.shape, 1, W.STAR, case.coeffs, W.BC_ZERO, "f32", method="tessellate")
    fused = Plan(case.shape, 1, W.STAR, case.coeffs, W.BC_ZERO, "f32", method="fused")
    ti, fi = tess.info(), fused.info()
    say("tessellated plan %s, fused plan %s" % (ti, fi))
    assert (ti["variant"], ti["fused_k"]) == (fi["variant"], fi["fused_k"])
    got = tess.run(x, case.T)
    ref = fused.run(x, case.T)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
