"""The tessellated tiling of Section 3.4 as the kernels schedule it, checked
on the CPU with a model of the iteration space (no GPU, no library).

The y axis is cut into tiles.  Stage A advances level j of a tile on its rows
[j r, h - j r) (a trapezoid: the triangle of the section's 1D figure); stage B
advances level j around every cut c on the rows [c - j r, c + j r) (the
inverted triangle).  The model pins three things the kernels rely on:
  * after stage A a tile of 2K+1 rows (r = 1) has the state pattern
    (0, 1, ..., K, ..., 1, 0), the section's (0,1,2,3,4,3,2,1,0) for K = 4;
  * stages A and B together compute every (row, level) exactly once: no
    redundant rows, no gaps, every row ends at level K;
  * every value stage B needs at level j-1 is either its own (computed at
    level j-1) or one of the 2r rows on each side of its valid region that
    stage A computed -- the slope rows the kernels store: rows [L r, (L+2) r)
    and [h - (L+2) r, h - L r) of a tile at level L.
"""
import itertools

import pytest


def stage_a_rows(h, K, r, j):
    return set(range(j * r, h - j * r))


def stage_b_rows(c, K, r, j):
    return set(range(c - j * r, c + j * r))


def tiles(n, Y, K, r):
    """Tile starts as the library cuts an axis of n rows into tiles of Y rows:
    a last tile shorter than 2(K+1)r shares the rows of the one before it."""
    need = 2 * (K + 1) * r
    count = -(-n // Y)
    starts = [t * Y for t in range(count)]
    if n - starts[-1] < need:
        a = starts[-2]
        starts[-1] = a + (n - a + 1) // 2
    ends = starts[1:] + [n]
    return list(zip(starts, ends))


@pytest.mark.parametrize("K", [1, 2, 3, 4, 5])
def test_triangle_state_pattern(K):
    h = 2 * K + 1
    state = [max((j for j in range(K + 1) if y in stage_a_rows(h, K, 1, j) or j == 0), default=0)
             for y in range(h)]
    assert state == [min(y, h - 1 - y) for y in range(h)]
    if K == 4:
        assert state == [0, 1, 2, 3, 4, 3, 2, 1, 0]   # the section's example


@pytest.mark.parametrize("n,Y,K,r,periodic", [(133, 64, 5, 1, False), (133, 64, 5, 1, True),
                                               (100, 64, 3, 1, False), (64, 64, 2, 2, True),
                                               (40, 64, 5, 1, True), (257, 32, 2, 2, False),
                                               (75, 16, 3, 1, True)])
def test_stages_cover_every_row_level_once(n, Y, K, r, periodic):
    ts = tiles(n, Y, K, r)
    assert all(b - a >= 2 * (K + 1) * r for a, b in ts)
    cuts = [a for a, _ in ts] + ([] if periodic else [n])
    count = {}
    for j in range(1, K + 1):
        for a, b in ts:
            for y in stage_a_rows(b - a, K, r, j):
                count[(a + y, j)] = count.get((a + y, j), 0) + 1
        for c in cuts:
            for y in stage_b_rows(c, K, r, j):
                if periodic:
                    y %= n
                elif not 0 <= y < n:
                    continue  # the zero halo: rows outside the grid stay 0
                count[(y, j)] = count.get((y, j), 0) + 1
    assert set(count) == set(itertools.product(range(n), range(1, K + 1)))
    assert set(count.values()) == {1}


@pytest.mark.parametrize("n,Y,K,r,periodic", [(133, 64, 5, 1, False), (100, 64, 3, 1, True),
                                               (257, 32, 2, 2, True), (64, 16, 2, 2, False)])
def test_stage_b_reads_only_own_rows_and_slopes(n, Y, K, r, periodic):
    ts = tiles(n, Y, K, r)
    # slope rows stage A stores, per level, in grid rows
    slopes = {L: set() for L in range(1, K)}
    for a, b in ts:
        h = b - a
        for L in range(1, K):
            assert set(range(L * r, (L + 2) * r)) <= stage_a_rows(h, K, r, L)
            assert set(range(h - (L + 2) * r, h - L * r)) <= stage_a_rows(h, K, r, L)
            slopes[L] |= {a + y for y in range(L * r, (L + 2) * r)}
            slopes[L] |= {a + y for y in range(h - (L + 2) * r, h - L * r)}
    cuts = [a for a, _ in ts] + ([] if periodic else [n])
    for c in cuts:
        for j in range(2, K + 1):
            own = stage_b_rows(c, K, r, j - 1)
            for y in stage_b_rows(c, K, r, j):
                for dy in range(-r, r + 1):
                    src = y + dy
                    if src in own:
                        continue
                    if periodic:
                        src %= n
                    elif not 0 <= src < n:
                        continue  # zero halo
                    assert src in slopes[j - 1], (c, j, y, dy)
