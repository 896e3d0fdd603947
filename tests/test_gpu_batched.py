"""GPU parity of the batched persistent sweep (stencil_batch_* / stencil_run_batched).

Every grid of a batch must equal its own single-grid sweep bit for bit (the
kernels share the per-point arithmetic), graph replays must all reproduce
that result, and a sample of grids is checked against the FP64 oracle.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import TOL, rel_err, say
from paper_2103_08825_amd import Plan
from paper_2103_08825_amd import workloads as W
from paper_2103_08825_amd._lib import StencilError
from paper_2103_08825_amd.batched import Batch, run_batched

pytestmark = pytest.mark.gpu


def _mixed_batch(seed, count, lo=17, hi=300, dt="f32"):
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(count):
        shape = (int(rng.integers(lo, hi)), int(rng.integers(lo, hi)))
        r = 1 if i % 3 else 2
        kind = int(rng.integers(0, 2))
        bc = int(rng.integers(0, 2))
        T = [0, 1, 3, 7, 10, 13, 22][i % 7]
        c = W.coefficients(rng, W.num_points(2, r, kind))
        u0 = rng.uniform(-1, 1, shape)
        specs.append((shape, r, kind, bc, T, c, u0))
    plans = [Plan(s[0], s[1], s[2], s[5], s[3], dt) for s in specs]
    xs = [torch.from_numpy(s[6]).to(plans[0].dtype).cuda() for s in specs]
    return specs, plans, xs


def test_single_pass_batch_equals_single_runs():
    """Every grid finishes in one pass (T <= k): no item waits for another."""
    specs, plans, xs = _mixed_batch(6, 12)
    Ts = [min(s[4], 3) for s in specs]
    ys = [torch.full_like(x, float("nan")) for x in xs]
    say("single-pass batch: launching")
    run_batched(plans, xs, ys, Ts)
    torch.cuda.synchronize()
    say("single-pass batch: done")
    for i, (p, x, y, T) in enumerate(zip(plans, xs, ys, Ts)):
        assert torch.equal(y, p.run(x, T)), i


@pytest.mark.parametrize("dt", ["f32", "f64", "bf16"])
def test_batch_equals_single_runs(dt):
    specs, plans, xs = _mixed_batch(1, 24, dt=dt)
    ys = [torch.full_like(x, float("nan")) for x in xs]
    say("batched %s: %d grids, launching" % (dt, len(plans)))
    run_batched(plans, xs, ys, [s[4] for s in specs])
    torch.cuda.synchronize()
    say("batched %s: done" % dt)
    for i, (s, p, x, y) in enumerate(zip(specs, plans, xs, ys)):
        ref = p.run(x, s[4])
        torch.cuda.synchronize()
        if dt == "bf16":
            # a batched pass may fuse a different number of steps than the plan
            err = float((y.double() - ref.double()).abs().max() / max(1e-30, float(ref.double().abs().max())))
            assert err <= TOL[dt], (i, s[:5], err)
        else:
            assert torch.equal(y, ref), (i, s[:5])


def test_batch_matches_oracle_sample():
    specs, plans, xs = _mixed_batch(2, 10, dt="f64")
    ys = [torch.empty_like(x) for x in xs]
    run_batched(plans, xs, ys, [s[4] for s in specs])
    torch.cuda.synchronize()
    for s, y in zip(specs, ys):
        shape, r, kind, bc, T, c, u0 = s
        ref = oracle.run(u0, c, T, r=r, kind=kind, bc=bc)
        assert rel_err(y.cpu().numpy(), ref) <= 1e-12


def test_graph_replays_reproduce_with_eager_work_between():
    specs, plans, xs = _mixed_batch(3, 16)
    ys = [torch.zeros_like(x) for x in xs]
    Ts = [s[4] for s in specs]
    b = Batch(plans, xs, ys, Ts)
    items, wgs = b.info()
    say("batch: %d items on %d workgroups" % (items, wgs))
    refs = []
    for p, x, T in zip(plans, xs, Ts):
        refs.append(p.run(x, T))
    torch.cuda.synchronize()
    for rep in range(4):
        for y in ys:
            y.fill_(float("nan"))          # eager work between replays
        b.launch()
        b.status()
        for i, (y, ref) in enumerate(zip(ys, refs)):
            assert torch.equal(y, ref), (rep, i)
        _ = plans[0].run(xs[0], 2)          # more eager work on the same stream
        torch.cuda.synchronize()
    b.close()


def test_batch_with_autotune_flag():
    specs, plans, xs = _mixed_batch(4, 6)
    ys = [torch.empty_like(x) for x in xs]
    b = Batch(plans, xs, ys, [s[4] for s in specs], autotune=True)
    b.launch()
    b.status()
    for s, p, x, y in zip(specs, plans, xs, ys):
        assert torch.equal(y, p.run(x, s[4]))
    b.close()


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_item_tuner_keeps_every_grid_equal_to_its_single_run(dt):
    """Flags bit 1: the depth and rows chosen by timing the batch's own replays
    change only the work split (FP32 and FP64 fused passes are bitwise equal to
    one-step sweeps), the choice lies in the searched sets, and a second batch of
    the same workload takes the cached choice."""
    specs, plans, xs = _mixed_batch(7, 14, dt=dt)
    Ts = [s[4] for s in specs]
    ys = [torch.full_like(x, float("nan")) for x in xs]
    say("item tuner %s: tuning" % dt)
    b = Batch(plans, xs, ys, Ts, tune_items=True)
    depths, chunk = b.choice()
    say("item tuner %s: depths %s, rows %d" % (dt, depths, chunk))
    assert depths[0] in (0, 6, 8, 10, 12) and depths[1] in (0, 6, 8, 10, 12)
    assert depths[2] in (0, 2, 3, 4) and depths[3] in (0, 2, 3, 4)
    assert chunk in (64, 96, 128, 192, 256)
    for y in ys:
        y.fill_(float("nan"))
    b.launch()
    b.status()
    for i, (p, x, y, T) in enumerate(zip(plans, xs, ys, Ts)):
        assert torch.equal(y, p.run(x, T)), i
    b2 = Batch(plans, xs, ys, Ts, tune_items=True)
    assert b2.choice() == (depths, chunk)
    b2.close()
    b.close()


def test_batch_argument_errors():
    specs, plans, xs = _mixed_batch(5, 3)
    ys = [torch.empty_like(x) for x in xs]
    p3 = Plan((8, 8, 8), 1, 0, [1 / 7] * 7, 0, "f32")
    x3 = torch.zeros((8, 8, 8), device="cuda")
    with pytest.raises(StencilError):
        run_batched([p3], [x3], [torch.empty_like(x3)], [3])
    with pytest.raises(StencilError):
        run_batched(plans[:1], xs[:1], xs[:1], [3])          # input aliases output
    pd = Plan(specs[0][0], specs[0][1], specs[0][2], specs[0][5], 0, "f64")
    with pytest.raises(StencilError):
        run_batched([plans[0], pd], [xs[0], xs[0].double()], [ys[0], torch.empty_like(xs[0]).double()], [2, 2])


def test_paper_scale_batch_equals_single_runs():
    """The uneven workload: 256 grids, sides log-uniform in [64, 2048], 5-point
    star or 9-point box, T uniform in [10, 200]; each grid against its own
    single-grid sweep (bitwise) and eight against the oracle on the whole field."""
    grids = W.batched_grids(seed=0)
    plans, xs = [], []
    for i, g in enumerate(grids):
        plans.append(Plan(g.shape, 1, g.kind, g.coeffs, W.BC_ZERO, "f32"))
        xs.append(torch.from_numpy(W.batched_field(0, g)).float().cuda())
    ys = [torch.empty_like(x) for x in xs]
    Ts = [g.T for g in grids]
    say("paper-scale batch: %d grids, %d points" % (len(grids), sum(x.numel() for x in xs)))
    b = Batch(plans, xs, ys, Ts)
    b.launch()
    b.status()
    torch.cuda.synchronize()
    for i, (p, x, y, T) in enumerate(zip(plans, xs, ys, Ts)):
        ref = p.run(x, T)
        torch.cuda.synchronize()
        assert torch.equal(y, ref), i
    # eight grids, whole fields, against the oracle at the FP32 tolerance
    rng = np.random.default_rng(0)
    for i in rng.choice(len(grids), size=8, replace=False):
        g = grids[i]
        u0 = xs[i].double().cpu().numpy()
        c32 = g.coeffs.astype(np.float32).astype(np.float64)
        ref = oracle.run(u0, c32, g.T, r=1, kind=g.kind, bc=W.BC_ZERO)
        err = rel_err(ys[i].double().cpu().numpy(), ref)
        say("  grid %d %s %s T=%d: rel err %.3e" % (i, g.shape, "box" if g.kind else "star", g.T, err))
        assert err <= 1e-5, (i, err)
    b.close()
    # the item tuner on the same workload: every grid bitwise equal to the default batch's
    ys2 = [torch.full_like(x, float("nan")) for x in xs]
    say("paper-scale batch: tuning the items")
    bt = Batch(plans, xs, ys2, Ts, tune_items=True)
    say("  tuned depths %s, rows %d" % bt.choice())
    for y in ys2:
        y.fill_(float("nan"))
    bt.launch()
    bt.status()
    for i, (y, y2) in enumerate(zip(ys, ys2)):
        assert torch.equal(y, y2), i
    bt.close()


def test_wait_limit_gives_up_and_the_next_replay_recovers():
    """A zero wait limit (set from the host) makes the first unsatisfied wait give
    up: the error flag makes every later wait of that replay give up at once, the
    kernel ends, and the batch reports a device error.  With the default limit
    restored the next replay clears the flag and completes."""
    rng = np.random.default_rng(9)
    c = W.coefficients(rng, 5)
    shape, T = (512, 512), 64  # 8 passes of 8 steps, dozens of items per pass
    plan = Plan(shape, 1, 0, c, 0, "f32")
    x = torch.from_numpy(rng.uniform(-1, 1, shape)).float().cuda()
    y = torch.empty_like(x)
    b = Batch([plan], [x], [y], [T])
    say("wait limit 0: launching")
    b.set_wait_limit(0)
    b.launch()
    with pytest.raises(StencilError):
        b.status()
    say("wait limit restored: launching")
    b.set_wait_limit(1_000_000)
    b.launch()
    b.status()
    torch.cuda.synchronize()
    assert torch.equal(y, plan.run(x, T))
    with pytest.raises(StencilError):
        b.set_wait_limit(-1)
    b.close()
