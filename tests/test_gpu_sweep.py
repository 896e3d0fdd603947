"""GPU parity of the sweep kernels against the FP64 oracle (small grids).

Grids span several output tiles and several z-chunks with ragged tails; every
compiled fused kernel family is run for k = 1, a middle k and the largest
compiled k, with T values that exercise the remainder pass (T mod k != 0).
Tolerances (normwise, max|gpu - oracle| / max|oracle|): 1e-12 FP64, 1e-5
FP32, 2e-2 BF16/FP16; power-of-two weights with small-integer fields make
every partial sum exact, so there the comparison is bitwise.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import TOL, TORCH, gpu_sweep, rel_err, rounded_inputs, say
from paper_2103_08825_amd import Plan, reduce
from paper_2103_08825_amd import _lib
from paper_2103_08825_amd import workloads as W

pytestmark = pytest.mark.gpu

SHAPES = {3: (21, 53, 131), 2: (45, 301), 1: (1003,)}
SHAPES_VX = {3: (13, 40, 128), 2: (37, 300), 1: (1000,)}   # last extent a multiple of 4
CHUNK = {3: 8, 2: 16, 1: 0}

# (dim, r, kind, dtype, kmax compiled for the default variant)
FAMILIES = [
    (3, 1, 0, "f32", 6), (3, 1, 1, "f32", 4), (3, 2, 0, "f32", 3),
    (3, 1, 0, "f64", 2), (3, 1, 1, "f64", 2), (3, 2, 0, "f64", 2),
    (2, 1, 0, "f32", 8), (2, 1, 1, "f32", 8), (2, 2, 0, "f32", 4), (2, 2, 1, "f32", 4),
    (2, 1, 0, "f64", 4), (2, 1, 1, "f64", 4), (2, 2, 0, "f64", 2),
    (1, 1, 0, "f64", 32), (1, 2, 0, "f64", 16), (1, 1, 0, "f32", 32), (1, 2, 0, "f32", 16),
]


def _case(dim, r, kind, bc, shape, seed):
    rng = np.random.default_rng(seed)
    c = W.coefficients(rng, W.num_points(dim, r, kind))
    u0 = rng.uniform(-1, 1, shape)
    return c, u0


def _check(dim, r, kind, bc, dt, shape, method, k, Ts, variant=0, seed=0):
    c, u0 = _case(dim, r, kind, bc, shape, seed)
    t_in, u_ex, c_ex = rounded_inputs(u0, c, dt)
    plan = Plan(shape, r, kind, c, bc, dt, method=method, fused_k=k, variant=variant,
                chunk=CHUNK[dim])
    info = plan.info()
    for T in Ts:
        say("case dim=%d r=%d kind=%d bc=%d %s shape=%s method=%s k=%d variant=%d T=%d" %
            (dim, r, kind, bc, dt, shape, method, info["fused_k"], info["variant"], T))
        got = gpu_sweep(plan, t_in, T)
        ref = oracle.run(u_ex, c_ex, T, r=r, kind=kind, bc=bc)
        err = rel_err(got, ref)
        assert err <= TOL[dt], "T=%d err=%.3e" % (T, err)
    plan.close()


@pytest.mark.parametrize("fam", FAMILIES, ids=lambda f: "%dd_r%d_%s_%s" % (f[0], f[1], "box" if f[2] else "star", f[3]))
@pytest.mark.parametrize("bc", [0, 1])
def test_fused_matches_oracle(fam, bc):
    dim, r, kind, dt, kmax = fam
    # 2D order-2 kernels are compiled with 4-column lanes only: width divisible by 4
    shape = SHAPES_VX[dim] if (dim == 2 and r == 2) else SHAPES[dim]
    for k in sorted({1, max(1, kmax // 2), kmax}):
        Ts = sorted({1, max(1, k - 1), k, k + 1, 2 * k + 1})
        _check(dim, r, kind, bc, dt, shape, "fused", k, Ts, seed=k)


@pytest.mark.parametrize("bc", [0, 1])
def test_2d_star_deepest_wide_lanes(bc):
    """The 2D 5-point star's deepest pass on 4-column lanes (the 8192^2 default
    depth), with remainders, against the oracle."""
    _check(2, 1, 0, bc, "f32", SHAPES_VX[2], "fused", 10, [3, 10, 11, 21], variant=2, seed=31)


@pytest.mark.parametrize("dim", [1, 2, 3])
@pytest.mark.parametrize("bc", [0, 1])
def test_wide_lane_variants(dim, bc):
    """Every compiled tile variant, on a shape whose last extent allows wide lanes."""
    nv = {3: 3, 2: 2, 1: 2}[dim]
    dt = "f64" if dim == 1 else "f32"   # 1D FP32 is compiled with wide lanes only
    for variant in range(1, nv + 1):
        _check(dim, 1, 0, bc, dt, SHAPES_VX[dim], "fused", 2, [1, 3, 5], variant=variant,
               seed=variant)


@pytest.mark.parametrize("dim,r,kind", [(3, 1, 0), (3, 1, 1), (3, 2, 0), (2, 1, 0), (2, 1, 1),
                                        (2, 2, 1), (1, 1, 0)])
@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_dyadic_bitwise(dim, r, kind, dt):
    """Exact inputs: the fused result, the plain result and the oracle agree bit for bit."""
    rng = np.random.default_rng(3)
    shape = SHAPES_VX[dim]
    c = W.dyadic_coefficients(dim, r, kind)
    u0 = W.dyadic_field(rng, shape)
    T = 3 if dt == "f32" else 5
    for bc in (0, 1):
        ref = oracle.run(u0, c, T, r=r, kind=kind, bc=bc)
        for method in ("fused", "plain", "generic"):
            say("dyadic dim=%d r=%d kind=%d bc=%d %s method=%s" % (dim, r, kind, bc, dt, method))
            plan = Plan(shape, r, kind, c, bc, dt, method=method, chunk=CHUNK[dim])
            got = gpu_sweep(plan, torch.from_numpy(u0).to(TORCH[dt]), T)
            np.testing.assert_array_equal(got, ref)
            plan.close()


@pytest.mark.parametrize("dim,r,kind", [(1, 1, 0), (1, 3, 0), (1, 4, 1), (2, 1, 0), (2, 3, 1),
                                        (2, 4, 0), (3, 1, 0), (3, 1, 1), (3, 2, 1), (3, 3, 0)])
@pytest.mark.parametrize("bc", [0, 1])
def test_generic_matches_oracle(dim, r, kind, bc):
    shape = {1: (97,), 2: (23, 29), 3: (9, 11, 13)}[dim]
    c, u0 = _case(dim, r, kind, bc, shape, 11)
    plan = Plan(shape, r, kind, c, bc, "f64", method="generic")
    say("generic dim=%d r=%d kind=%d bc=%d" % (dim, r, kind, bc))
    got = gpu_sweep(plan, torch.from_numpy(u0), 4)
    ref = oracle.run(u0, c, 4, r=r, kind=kind, bc=bc)
    assert rel_err(got, ref) <= 1e-12


@pytest.mark.parametrize("fam", [(3, 1, 0), (3, 1, 1), (3, 2, 0), (2, 1, 0), (2, 1, 1), (2, 2, 0),
                                 (1, 1, 0)])
@pytest.mark.parametrize("dt", ["bf16", "f16"])
def test_low_precision(fam, dt):
    dim, r, kind = fam
    shape = SHAPES_VX[dim]
    for bc in (0, 1):
        for k in (1, 2):
            _check(dim, r, kind, bc, dt, shape, "fused", k, [1, 4, 7], seed=5)


def test_small_grids_and_degenerate_extents():
    """Grids smaller than one tile, extents of 1, and periodic extents below the radius."""
    for shape, r, kind, bc in [((1, 1, 1), 1, 0, 0), ((1, 1, 1), 1, 1, 1), ((2, 3, 5), 2, 0, 1),
                               ((3, 1, 7), 1, 1, 0), ((1, 9), 1, 1, 1), ((4, 1), 2, 0, 1),
                               ((1,), 1, 0, 0), ((3,), 2, 0, 1)]:
        dim = len(shape)
        c, u0 = _case(dim, r, kind, bc, shape, 2)
        for method in ("auto", "generic"):
            say("tiny shape=%s r=%d kind=%d bc=%d %s" % (shape, r, kind, bc, method))
            plan = Plan(shape, r, kind, c, bc, "f64", method=method)
            got = gpu_sweep(plan, torch.from_numpy(u0), 5)
            ref = oracle.run(u0, c, 5, r=r, kind=kind, bc=bc)
            assert rel_err(got, ref) <= 1e-12, (shape, method)
            plan.close()


def test_T_zero_copies_and_aliasing():
    shape = SHAPES[3]
    c, u0 = _case(3, 1, 0, 0, shape, 4)
    plan = Plan(shape, 1, 0, c, 0, "f32", fused_k=3)
    x = torch.from_numpy(u0).float().cuda()
    out = plan.run(x, 0)
    torch.cuda.synchronize()
    assert torch.equal(out, x)
    ref = plan.run(x, 7).clone()
    y = x.clone()
    plan.run(y, 7, out=y)            # in place: d_in == d_out
    torch.cuda.synchronize()
    assert torch.equal(y, ref)


def test_unaligned_buffers_fall_back():
    """A view at an odd element offset cannot use wide-lane loads; results must not change."""
    shape = SHAPES_VX[2]
    c, u0 = _case(2, 1, 1, 1, shape, 6)
    plan = Plan(shape, 1, 1, c, 1, "f32", fused_k=4, variant=2)
    base = torch.zeros(u0.size + 1, dtype=torch.float32, device="cuda")
    view = base[1:].view(shape)
    view.copy_(torch.from_numpy(u0).float())
    outb = torch.zeros_like(base)
    out = outb[1:].view(shape)
    plan.run(view, 6, out=out)
    ref = plan.run(view.contiguous().clone(), 6)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)


def test_plan_info_and_autotune():
    shape = (24, 40, 128)
    c, u0 = _case(3, 1, 0, 0, shape, 8)
    plan = Plan(shape, 1, 0, c, 0, "f32", autotune=True)
    x = torch.from_numpy(u0).float().cuda()
    got = plan.run(x, 9)
    torch.cuda.synchronize()
    info = plan.info()
    say("autotuned:", info)
    assert info["tuned"] == 1 and info["method"] == _lib.METHOD_FUSED
    ref = oracle.run(x.double().cpu().numpy(), c.astype(np.float32).astype(np.float64), 9, r=1,
                     kind=0, bc=0)
    assert rel_err(got.double().cpu().numpy(), ref) <= 1e-5


@pytest.mark.parametrize("dt", ["f64", "f32", "bf16", "f16"])
def test_fp64_reductions(dt):
    rng = np.random.default_rng(9)
    for n in (0, 1, 1000, 1 << 20, (1 << 20) + 37):
        a = torch.from_numpy(rng.uniform(-1, 1, n)).to(TORCH[dt]).cuda()
        b = torch.from_numpy(rng.uniform(-1, 1, n)).to(TORCH[dt]).cuda()
        got = reduce(a, b).cpu().numpy()
        x, y = a.double().cpu().numpy(), b.double().cpu().numpy()
        if n == 0:
            np.testing.assert_array_equal(got, np.zeros(6))
            continue
        ref = [x.sum(), (x * x).sum(), np.abs(x).max(), ((x - y) ** 2).sum(),
               np.abs(x - y).max(), np.abs(y).max()]
        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-9)
        got1 = reduce(a).cpu().numpy()
        np.testing.assert_allclose(got1[:3], ref[:3], rtol=1e-12, atol=1e-9)
        assert (got1[3:] == 0).all()
        # deterministic
        assert np.array_equal(reduce(a, b).cpu().numpy(), got)


def test_fp64_reductions_unaligned():
    rng = np.random.default_rng(10)
    n = 10007
    base = torch.from_numpy(rng.uniform(-1, 1, n + 1)).float().cuda()
    a = base[1:]
    got = reduce(a).cpu().numpy()
    x = a.double().cpu().numpy()
    np.testing.assert_allclose(got[:3], [x.sum(), (x * x).sum(), np.abs(x).max()], rtol=1e-12)


@pytest.mark.parametrize("dim,r,kind,dt", [(3, 1, 0, "f32"), (3, 1, 1, "f32"), (3, 2, 0, "f64"),
                                           (2, 1, 1, "f32"), (2, 2, 0, "f32"), (1, 1, 0, "f64"),
                                           (3, 1, 0, "bf16")])
@pytest.mark.parametrize("bc", [0, 1])
def test_fused_plain_generic_bitwise_on_random_inputs(dim, r, kind, dt, bc):
    """Every kernel accumulates a point's terms in the same order with the same
    fused multiply-adds, so all methods agree bit for bit on any input -- except
    that with 16-bit storage a fused pass keeps its intermediate steps in FP32
    (rounding only on the store), so there only plain and generic coincide."""
    shape = SHAPES_VX[dim]
    c, u0 = _case(dim, r, kind, bc, shape, 12)
    x = torch.from_numpy(u0).to(TORCH[dt]).cuda()
    outs = {}
    for method in ("fused", "plain", "generic"):
        say("bitwise dim=%d r=%d kind=%d %s bc=%d %s" % (dim, r, kind, dt, bc, method))
        p = Plan(shape, r, kind, c, bc, dt, method=method, chunk=CHUNK[dim])
        outs[method] = p.run(x, 7)
        torch.cuda.synchronize()
    assert torch.equal(outs["plain"], outs["generic"])
    if dt in ("f32", "f64"):
        assert torch.equal(outs["fused"], outs["plain"])
    else:
        ref = outs["plain"].double()
        assert float((outs["fused"].double() - ref).abs().max() / ref.abs().max()) <= TOL[dt]


@pytest.mark.parametrize("method", ["plain", "fused"])
def test_graph_replays_match_eager_runs(method):
    """Recorded launches (graph=True) replay the same sweep as eager runs, bit for
    bit, on every replay, with eager work on the stream between replays; a new
    (input, output, T) triple re-records; an aliased input still works."""
    case = W.case_1d3p(seed=3, n=4099, T=37)
    x = torch.from_numpy(case.u0).cuda()
    eager = Plan(case.shape, 1, W.STAR, case.coeffs, W.BC_ZERO, "f64", method=method)
    graph = Plan(case.shape, 1, W.STAR, case.coeffs, W.BC_ZERO, "f64", method=method, graph=True)
    ref = eager.run(x, case.T)
    y = torch.empty_like(x)
    for rep in range(4):
        y.fill_(float("nan"))
        graph.run(x, case.T, out=y)
        _ = eager.run(x, 5)                          # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(y, ref), rep
    ref2 = eager.run(x, 12)
    graph.run(x, 12, out=y)                          # new triple: re-recorded
    torch.cuda.synchronize()
    assert torch.equal(y, ref2)
    z = x.clone()
    graph.run(z, case.T, out=z)                      # aliased input and output
    torch.cuda.synchronize()
    assert torch.equal(z, ref)
    for T, r in ((case.T, ref), (12, ref2)):
        want = oracle.run(case.u0, case.coeffs, T, r=1, kind=W.STAR, bc=W.BC_ZERO)
        assert rel_err(r.cpu().numpy(), want) <= 1e-12
    # a 3D fused plan records its passes the same way
    c3 = W.case_3d("3d7p", seed=1, n=40, T=11)
    x3 = torch.from_numpy(c3.u0).float().cuda()
    g3 = Plan(c3.shape, 1, W.STAR, c3.coeffs, W.BC_ZERO, "f32", method="fused", graph=True)
    e3 = Plan(c3.shape, 1, W.STAR, c3.coeffs, W.BC_ZERO, "f32", method="fused")
    y3 = torch.empty_like(x3)
    for rep in range(3):
        g3.run(x3, c3.T, out=y3)
        torch.cuda.synchronize()
        assert torch.equal(y3, e3.run(x3, c3.T)), rep


# tile shapes (columns per lane, waves, rows per wave) of the 3D variant ids
V3 = {1: (1, 4, 8), 2: (1, 8, 8), 3: (2, 4, 8), 4: (1, 8, 4), 5: (1, 16, 4), 6: (2, 8, 4)}
INTERIOR_SHAPE = (40, 140, 256)


def _unmasked_workgroups(shape, r, k, variant, tile):
    """Workgroups of a zero-halo 3D launch whose widened tile and every plane
    their outputs depend on lie inside the grid: the ones that take the
    kernel's path without per-point boundary masks."""
    n0, n1, n2 = shape
    vx, nw, rw = V3[variant]
    out_x, out_y, chunk = tile
    halo_x = -(-k * r // vx) * vx
    count = 0
    for zc in range(-(-n0 // chunk)):
        z0, z1 = zc * chunk, min(zc * chunk + chunk, n0)
        if z0 - k * r < 0 or z1 + k * r > n0:
            continue
        for ty in range(-(-n1 // out_y)):
            yb = ty * out_y - k * r
            if yb < 0 or yb + nw * rw > n1:
                continue
            for tx in range(-(-n2 // out_x)):
                xb = tx * out_x - halo_x
                if 0 <= xb and xb + 64 * vx <= n2:
                    count += 1
    return count


@pytest.mark.parametrize("dt", ["f32", "bf16", "f16", "f64"])
@pytest.mark.parametrize("name", ["3d7p", "3d27p", "3d13p"])
def test_default_tiles_on_interior_reaching_grid(name, dt):
    """The 512^3 defaults (tile variant and fused depth of every stencil and
    storage type, and the plain comparator's tile) on a grid with tiles that lie
    wholly inside it, so that the unmasked zero-halo path runs next to the
    masked one; element-wise against the oracle, with a remainder pass."""
    big = W.case_3d(name, seed=0, n=8, T=1)   # only its stencil and weights
    ref_plan = Plan((512, 512, 512), big.r, big.kind, big.coeffs, W.BC_ZERO, dt)
    info512 = ref_plan.info()
    ref_plan.close()
    rng = np.random.default_rng(17)
    u0 = rng.uniform(-1, 1, INTERIOR_SHAPE)
    t_in, u_ex, c_ex = rounded_inputs(u0, big.coeffs, dt)
    runs = [("fused", info512["variant"], info512["fused_k"])]
    if dt == "f32":
        pl = Plan((512, 512, 512), big.r, big.kind, big.coeffs, W.BC_ZERO, dt, method="plain")
        runs.append(("plain", pl.info()["variant"], 1))
        pl.close()
    for method, variant, k in runs:
        plan = Plan(INTERIOR_SHAPE, big.r, big.kind, big.coeffs, W.BC_ZERO, dt, method=method,
                    fused_k=k if method == "fused" else 0, variant=variant, chunk=8)
        info = plan.info()
        assert (info["variant"], info["fused_k"]) == (variant, k)
        inner = _unmasked_workgroups(INTERIOR_SHAPE, big.r, k, variant, info["tile"])
        assert inner > 0, info
        T = 2 * k + 1
        say("interior %s %s %s variant=%d k=%d tile=%s T=%d (%d unmasked workgroups)"
            % (name, dt, method, variant, k, info["tile"], T, inner))
        got = gpu_sweep(plan, t_in, T)
        ref = oracle.run(u_ex, c_ex, T, r=big.r, kind=big.kind, bc=W.BC_ZERO)
        err = rel_err(got, ref)
        say("  rel err %.3e" % err)
        assert err <= TOL[dt]
        plan.close()
