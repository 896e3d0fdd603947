"""Pin the FP64 oracle to results fixed by the paper's definition and by mathematics.

Every test here runs on the CPU.  None compares the oracle with itself: each
checks it against a hand-worked fixture, a closed form (DFT, DST-I), an
independent library filter (scipy.ndimage), or an exact invariant.  The
mistakes these are chosen to catch: a mirrored offset (x - o instead of x + o),
a wrong canonical order, a dropped or duplicated term, a wrong boundary rule,
a wrong axis order, a wrong adjoint direction.
"""
import json
import os

import numpy as np
import pytest

import oracle
import pins
from paper_2103_08825_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
STENCILS = [(1, 1, 0), (1, 2, 0), (1, 1, 1), (2, 1, 0), (2, 1, 1), (2, 2, 0), (2, 2, 1),
            (3, 1, 0), (3, 1, 1), (3, 2, 0)]


def test_canonical_offsets_match_golden():
    with open(os.path.join(GOLDEN, "canonical_offsets.json")) as f:
        data = json.load(f)
    for case in data["cases"]:
        got = oracle.offsets(case["dim"], case["r"], case["kind"])
        assert got.tolist() == case["offsets"], case["name"]
        assert oracle.num_points(case["dim"], case["r"], case["kind"]) == len(case["offsets"])


@pytest.mark.parametrize("dim,r,kind", STENCILS + [(3, 3, 1), (2, 4, 1), (3, 4, 0)])
def test_offset_set_properties(dim, r, kind):
    offs = oracle.offsets(dim, r, kind)
    n = 2 * dim * r + 1 if kind == 0 else (2 * r + 1) ** dim
    assert offs.shape == (n, dim)
    assert len({tuple(o) for o in offs}) == n                      # no duplicates
    assert np.abs(offs).max() == r
    if kind == 0:
        assert all(np.count_nonzero(o) <= 1 for o in offs)
    # symmetric set, and negation reverses the canonical order
    assert (offs[::-1] == -offs).all()
    # lexicographic order
    keys = [tuple(o) for o in offs]
    assert keys == sorted(keys)


def test_bad_arguments_rejected():
    assert oracle.num_points(0, 1, 0) == -1
    assert oracle.num_points(4, 1, 0) == -1
    assert oracle.num_points(2, 0, 0) == -1
    assert oracle.num_points(2, 1, 2) == -1
    with pytest.raises(ValueError):
        oracle.run(np.zeros(4), [1.0, 0.0], 1, r=1, kind=0, bc=0)


def test_hand_examples():
    with open(os.path.join(GOLDEN, "hand_examples.json")) as f:
        data = json.load(f)
    for case in data["cases"]:
        u0 = np.array(case["u0"], dtype=np.float64)
        got = oracle.run(u0, case["coeffs"], case["T"], r=case["r"], kind=case["kind"],
                         bc=case["bc"])
        np.testing.assert_array_equal(got, np.array(case["uT"], dtype=np.float64),
                                      err_msg=case["name"])


def test_T_zero_is_identity():
    u = np.random.default_rng(1).uniform(-1, 1, (5, 6))
    out = oracle.run(u, W.coefficients(np.random.default_rng(2), 5), 0, r=1, kind=0, bc=0)
    np.testing.assert_array_equal(out, u)


@pytest.mark.parametrize("dim,r,kind", STENCILS)
@pytest.mark.parametrize("bc", [0, 1])
def test_matches_ndimage_correlate(dim, r, kind, bc):
    """scipy's correlation filter, applied T times, with random non-symmetric weights."""
    rng = np.random.default_rng(100 + dim * 10 + r * 3 + kind + 7 * bc)
    shape = {1: (23,), 2: (9, 11), 3: (6, 7, 5)}[dim]
    c = W.coefficients(rng, oracle.num_points(dim, r, kind))
    u0 = rng.uniform(-1, 1, shape)
    T = 4
    ref = pins.ndimage_sweep(u0, pins.canonical_offsets(dim, r, kind), c, r, bc, T)
    got = oracle.run(u0, c, T, r=r, kind=kind, bc=bc)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-14)


@pytest.mark.parametrize("dim,r,kind", STENCILS)
def test_periodic_matches_fft_closed_form(dim, r, kind):
    rng = np.random.default_rng(7 + dim + 3 * r + 11 * kind)
    shape = {1: (64,), 2: (16, 12), 3: (8, 6, 10)}[dim]
    c = W.coefficients(rng, oracle.num_points(dim, r, kind))
    u0 = rng.uniform(-1, 1, shape)
    T = 9
    ref = pins.fft_sweep(u0, pins.canonical_offsets(dim, r, kind), c, T)
    got = oracle.run(u0, c, T, r=r, kind=kind, bc=1)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13)


def test_periodic_aliasing_when_radius_exceeds_extent():
    """r >= N: aliased terms are all summed (periodic rule applied per term)."""
    rng = np.random.default_rng(5)
    for shape, r in [((3,), 2), ((2, 5), 2), ((1, 3, 4), 1)]:
        dim = len(shape)
        c = W.coefficients(rng, oracle.num_points(dim, r, 1))
        u0 = rng.uniform(-1, 1, shape)
        ref = pins.fft_sweep(u0, pins.canonical_offsets(dim, r, 1), c, 3)
        got = oracle.run(u0, c, 3, r=r, kind=1, bc=1)
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-14)


def _symmetric_coeffs(offs, rng):
    """Weights depending only on |o_i| per axis (symmetric under each axis reflection)."""
    table = {}
    out = []
    for o in offs:
        key = tuple(abs(int(v)) for v in o)
        if key not in table:
            table[key] = rng.uniform(0.5, 1.5)
        out.append(table[key])
    out = np.array(out)
    return out / out.sum()


@pytest.mark.parametrize("dim,kind", [(1, 0), (2, 0), (2, 1), (3, 0), (3, 1)])
def test_zero_halo_matches_dst_closed_form(dim, kind):
    rng = np.random.default_rng(40 + dim + kind)
    shape = {1: (50,), 2: (13, 17), 3: (7, 9, 8)}[dim]
    offs = pins.canonical_offsets(dim, 1, kind)
    c = _symmetric_coeffs(offs, rng)
    u0 = rng.uniform(-1, 1, shape)
    T = 12
    ref = pins.dst_sweep(u0, offs, c, T)
    got = oracle.run(u0, c, T, r=1, kind=kind, bc=0)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13)


def test_1d_sine_mode_decays_by_eigenvalue():
    """A single zero-halo eigenmode of the symmetric 1D3P stencil is scaled by lambda^T."""
    n, m, T = 101, 7, 30
    a, b = 0.3, 0.4
    i = np.arange(n)
    v = np.sin(np.pi * m * (i + 1) / (n + 1))
    lam = b + 2 * a * np.cos(np.pi * m / (n + 1))
    got = oracle.run(v, [a, b, a], T, r=1, kind=0, bc=0)
    np.testing.assert_allclose(got, lam ** T * v, rtol=0, atol=1e-14)


@pytest.mark.parametrize("dim,r,kind", STENCILS)
def test_impulse_response_is_mirrored_pattern(dim, r, kind):
    """A unit impulse at x0 gives u_1[x0 - o_j] = c_j: pins direction and order."""
    shape = (2 * r + 3,) * dim
    x0 = np.array([r + 1] * dim)
    u0 = np.zeros(shape)
    u0[tuple(x0)] = 1.0
    n = oracle.num_points(dim, r, kind)
    c = np.arange(1, n + 1, dtype=np.float64)          # distinct weights
    got = oracle.run(u0, c, 1, r=r, kind=kind, bc=0)
    expect = np.zeros(shape)
    for o, cj in zip(pins.canonical_offsets(dim, r, kind), c):
        expect[tuple(x0 - o)] = cj
    np.testing.assert_array_equal(got, expect)


@pytest.mark.parametrize("dim,r,kind", STENCILS)
def test_dyadic_inputs_are_exact(dim, r, kind):
    """Power-of-two weights and small-integer fields: every partial sum is exact,
    so any summation order gives the same bits; compare with scipy bitwise."""
    rng = np.random.default_rng(3)
    shape = {1: (40,), 2: (10, 9), 3: (6, 5, 7)}[dim]
    c = W.dyadic_coefficients(dim, r, kind)
    assert c.sum() == 1.0
    u0 = W.dyadic_field(rng, shape)
    for bc in (0, 1):
        ref = pins.ndimage_sweep(u0, pins.canonical_offsets(dim, r, kind), c, r, bc, 3)
        got = oracle.run(u0, c, 3, r=r, kind=kind, bc=bc)
        np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("dim,r,kind", STENCILS)
def test_constant_field_preserved_periodic(dim, r, kind):
    shape = {1: (17,), 2: (7, 8), 3: (5, 4, 6)}[dim]
    c = W.dyadic_coefficients(dim, r, kind)
    u0 = np.full(shape, 3.0)
    got = oracle.run(u0, c, 10, r=r, kind=kind, bc=1)
    np.testing.assert_array_equal(got, u0)


@pytest.mark.parametrize("dim,r,kind", [(1, 1, 0), (2, 1, 1), (3, 1, 0), (3, 2, 0), (3, 1, 1)])
def test_affine_field_on_interior_cone(dim, r, kind):
    """u0 = a.x + b with sum c = 1 gives u_T = a.(x + T m1) + b away from the faces,
    m1 = sum_j c_j o_j (zero for symmetric weights, so a linear field is kept)."""
    rng = np.random.default_rng(9)
    shape = {1: (30,), 2: (20, 22), 3: (16, 15, 17)}[dim]
    offs = pins.canonical_offsets(dim, r, kind)
    n = len(offs)
    c = np.zeros(n)
    # dyadic, non-symmetric weights summing to 1
    c[:] = 1.0 / 64
    c[n // 2] = 1.0 - (n - 1) / 64
    c[0] += 1.0 / 16
    c[n // 2] -= 1.0 / 16
    assert c.sum() == 1.0
    a = rng.integers(-3, 4, size=dim).astype(np.float64)
    b = 5.0
    grids = np.meshgrid(*[np.arange(s, dtype=np.float64) for s in shape], indexing="ij")
    u0 = b + sum(ai * g for ai, g in zip(a, grids))
    T = 3
    got = oracle.run(u0, c, T, r=r, kind=kind, bc=0)
    m1 = (c[:, None] * offs).sum(axis=0)
    expect = b + sum(ai * (g + T * mi) for ai, g, mi in zip(a, grids, m1))
    inner = tuple(slice(T * r, s - T * r) for s in shape)
    np.testing.assert_allclose(got[inner], expect[inner], rtol=0, atol=1e-12)
    # symmetric weights keep a linear field exactly on the interior
    cs = W.dyadic_coefficients(dim, r, kind)
    got = oracle.run(u0, cs, T, r=r, kind=kind, bc=0)
    np.testing.assert_array_equal(got[inner], u0[inner])


@pytest.mark.parametrize("dim,r,kind", [(1, 1, 0), (2, 1, 1), (3, 1, 0), (3, 2, 0)])
def test_conservation_and_max_norm(dim, r, kind):
    rng = np.random.default_rng(12)
    shape = {1: (33,), 2: (12, 10), 3: (7, 8, 6)}[dim]
    c = W.coefficients(rng, oracle.num_points(dim, r, kind))
    u = rng.uniform(-1, 1, shape)
    s0 = u.sum()
    for _ in range(5):
        nxt = oracle.run(u, c, 1, r=r, kind=kind, bc=1)
        assert abs(nxt.sum() - s0) <= 1e-12 * u.size
        assert np.abs(nxt).max() <= np.abs(u).max() * (1 + 1e-15)
        z = oracle.run(u, c, 1, r=r, kind=kind, bc=0)
        assert np.abs(z).max() <= np.abs(u).max() * (1 + 1e-15)
        u = nxt


def test_block_run_matches_full_grid():
    rng = np.random.default_rng(21)
    for dim, r, kind, bc, shape, T in [(2, 1, 0, 0, (40, 37), 5), (2, 1, 1, 1, (30, 33), 4),
                                       (3, 2, 0, 0, (14, 15, 16), 2), (3, 1, 0, 1, (12, 13, 11), 3),
                                       (1, 1, 0, 1, (50,), 30)]:
        c = W.coefficients(rng, oracle.num_points(dim, r, kind))
        u0 = rng.uniform(-1, 1, shape)
        full = oracle.run(u0, c, T, r=r, kind=kind, bc=bc)
        for start, size in [((0,) * dim, (3,) * dim),
                            (tuple(s // 2 for s in shape), (2,) * dim),
                            (tuple(s - 4 for s in shape), (4,) * dim)]:
            blk = oracle.block_run(u0, c, T, start, size, r=r, kind=kind, bc=bc)
            sl = tuple(slice(a, a + b) for a, b in zip(start, size))
            np.testing.assert_array_equal(blk, full[sl])


# --- adjoint ---------------------------------------------------------------

@pytest.mark.parametrize("dim,r,kind,bc", [(1, 1, 0, 0), (1, 2, 0, 1), (2, 1, 1, 0),
                                           (2, 1, 0, 1), (3, 1, 0, 0), (3, 1, 1, 1),
                                           (3, 2, 0, 0)])
def test_adjoint_dot_product_identity(dim, r, kind, bc):
    """<A u, w> = <u, A^T w> with A = T forward steps and A^T the adjoint sweep."""
    rng = np.random.default_rng(30 + dim + r + kind + bc)
    shape = {1: (29,), 2: (9, 10), 3: (6, 7, 5)}[dim]
    c = W.coefficients(rng, oracle.num_points(dim, r, kind))
    u = rng.uniform(-1, 1, shape)
    w = rng.uniform(-1, 1, shape)
    T = 7
    Au = oracle.run(u, c, T, r=r, kind=kind, bc=bc)
    ATw, _ = oracle.adjoint(u, c, w, T, r=r, kind=kind, bc=bc, ckpt=3)
    lhs, rhs = np.vdot(Au, w), np.vdot(u, ATw)
    assert abs(lhs - rhs) <= 1e-13 * max(1.0, abs(lhs))


@pytest.mark.parametrize("dim,r,kind", [(1, 1, 0), (2, 1, 1), (3, 1, 0), (3, 2, 0)])
def test_adjoint_matches_fft_closed_form(dim, r, kind):
    rng = np.random.default_rng(50 + dim + r + kind)
    shape = {1: (32,), 2: (10, 12), 3: (6, 8, 7)}[dim]
    c = W.coefficients(rng, oracle.num_points(dim, r, kind))
    u0 = rng.uniform(-1, 1, shape)
    y = rng.uniform(-1, 1, shape)
    T = 6
    uT = oracle.run(u0, c, T, r=r, kind=kind, bc=1)
    g = uT - y
    gu, gc = oracle.adjoint(u0, c, g, T, r=r, kind=kind, bc=1, ckpt=4)
    ref_u, ref_c = pins.fft_adjoint(u0, g, pins.canonical_offsets(dim, r, kind), c, T)
    np.testing.assert_allclose(gu, ref_u, rtol=0, atol=1e-12)
    np.testing.assert_allclose(gc, ref_c, rtol=1e-11, atol=1e-11)


@pytest.mark.parametrize("bc", [0, 1])
def test_adjoint_coefficient_gradient_central_differences(bc):
    """L = 0.5 ||u_T - y||^2; dL/dc_j against central differences in c_j."""
    rng = np.random.default_rng(77 + bc)
    dim, r, kind, shape, T = 2, 1, 1, (8, 9), 5
    c = W.coefficients(rng, oracle.num_points(dim, r, kind))
    u0 = rng.uniform(-1, 1, shape)
    y = rng.uniform(-1, 1, shape)

    def loss(cc):
        return 0.5 * np.sum((oracle.run(u0, cc, T, r=r, kind=kind, bc=bc) - y) ** 2)

    uT = oracle.run(u0, c, T, r=r, kind=kind, bc=bc)
    gu, gc = oracle.adjoint(u0, c, uT - y, T, r=r, kind=kind, bc=bc, ckpt=2)
    h = 1e-5
    for j in range(len(c)):
        e = np.zeros_like(c)
        e[j] = h
        fd = (loss(c + e) - loss(c - e)) / (2 * h)
        assert abs(fd - gc[j]) <= 1e-6 * max(1.0, abs(gc[j]))
    # L is quadratic in u0: central differences along a direction are exact up to rounding
    d = rng.uniform(-1, 1, shape)
    h = 1e-3
    fd = (0.5 * np.sum((oracle.run(u0 + h * d, c, T, r=r, kind=kind, bc=bc) - y) ** 2)
          - 0.5 * np.sum((oracle.run(u0 - h * d, c, T, r=r, kind=kind, bc=bc) - y) ** 2)) / (2 * h)
    assert abs(fd - np.vdot(gu, d)) <= 1e-9 * max(1.0, abs(fd))


def test_adjoint_checkpoint_interval_invariance():
    rng = np.random.default_rng(88)
    shape, T = (6, 7, 8), 11
    c = W.coefficients(rng, 7)
    u0 = rng.uniform(-1, 1, shape)
    g = rng.uniform(-1, 1, shape)
    ref_u, ref_c = oracle.adjoint(u0, c, g, T, r=1, kind=0, bc=0, ckpt=1, nthreads=1)
    for ck in (2, 5, 11, 50):
        gu, gc = oracle.adjoint(u0, c, g, T, r=1, kind=0, bc=0, ckpt=ck, nthreads=1)
        np.testing.assert_array_equal(gu, ref_u)
        np.testing.assert_array_equal(gc, ref_c)


def test_adjoint_T_zero():
    u0 = np.ones((4, 5))
    g = np.arange(20.0).reshape(4, 5)
    gu, gc = oracle.adjoint(u0, W.coefficients(np.random.default_rng(0), 5), g, 0, r=1,
                            kind=0, bc=0)
    np.testing.assert_array_equal(gu, g)
    np.testing.assert_array_equal(gc, np.zeros(5))


def test_planted_mistakes_are_caught():
    """A mirrored offset set (x - o instead of x + o) or a reversed coefficient
    order must fail the pins above; check that the pins can tell."""
    rng = np.random.default_rng(4)
    c = W.coefficients(rng, 7)
    u0 = rng.uniform(-1, 1, (6, 7, 8))
    offs = pins.canonical_offsets(3, 1, 0)
    ref = pins.fft_sweep(u0, offs, c, 3)
    mirrored = pins.fft_sweep(u0, -offs, c, 3)
    reversed_c = pins.fft_sweep(u0, offs, c[::-1], 3)
    good = oracle.run(u0, c, 3, r=1, kind=0, bc=1)
    assert np.abs(good - ref).max() < 1e-13
    assert np.abs(mirrored - ref).max() > 1e-3
    assert np.abs(reversed_c - ref).max() > 1e-3
