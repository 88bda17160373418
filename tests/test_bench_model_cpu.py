"""The trailing-update launch model of bench.py (its roofline's flops and
bytes) against the LU's trailing work, counted tile by tile (no GPU)."""
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def _schedule(npan, group):
    """The trailing-update launches of one factorization as sets of (source
    panel, row tile, column tile) products, written from the scheme: singly,
    panel p updates every tile beyond it; in a group of g panels (g0 .. g0+g-1),
    after panel p the group's panels so far update the next panel's column of
    tiles and (groups of four) its row of tiles beyond it, and after the last the
    group updates every tile beyond the group; pairs leave the second panel's row
    of tiles to its pre-update (returned apart)."""
    launches, pre = [], set()
    for p in range(npan):
        g0 = p // group * group
        full = group > 1 and g0 + group <= npan and not (group == 2 and p + 2 > npan and p % 2 == 0)
        if group == 2:
            full = (p % 2 == 0 and p + 2 < npan) or (p % 2 == 1 and p + 1 < npan)
            g0 = p - p % 2
        j = p - g0 if full else -1
        srcs = range(g0, p + 1) if full else [p]
        if full and j < group - 1:
            nxt = p + 1
            t = {(q, i, nxt) for q in srcs for i in range(nxt, npan)}
            rows = {(q, nxt, c) for q in srcs for c in range(nxt + 1, npan)}
            if group == 4:
                t |= rows
            else:
                pre |= rows
            launches.append(t)
        elif full:
            launches.append({(q, i, c) for q in srcs for i in range(p + 1, npan) for c in range(p + 1, npan)})
        elif p + 1 < npan:
            launches.append({(p, i, c) for i in range(p + 1, npan) for c in range(p + 1, npan)})
    return [l for l in launches if l], pre


@pytest.mark.parametrize("npad", [512, 768, 1024, 2048])
@pytest.mark.parametrize("group", [1, 2, 4])
def test_update_launches_cover_the_trailing_work_once(npad, group):
    nb = 128
    npan = npad // nb
    launches, pre = _schedule(npan, group)
    seen = {}
    for l in launches + [pre]:
        for x in l:
            seen[x] = seen.get(x, 0) + 1
    # every product of panel q on a tile beyond it, exactly once
    want = {(q, i, c) for q in range(npan) for i in range(q + 1, npan) for c in range(q + 1, npan)}
    assert set(seen) == want and set(seen.values()) == {1}
    model = bench._update_launches(npad, nb, group)
    assert len(model) == len(launches)
    tile_flops = 2.0 * nb ** 3
    for (fl, _), l in zip(model, launches):
        assert fl == pytest.approx(tile_flops * len(l))
    total = sum(f for f, _ in model) + tile_flops * len(pre)
    assert total == pytest.approx(sum(2.0 * nb * (npad - (p + 1) * nb) ** 2 for p in range(npan)))


def test_update_launch_bytes_of_a_group_of_four():
    """A K = 512 launch moves A22 twice and its L and U blocks once; a group's
    L-shaped launch the column of tiles and the row of tiles twice, and its L
    rows and U columns once."""
    nb, npad = 128, 1024
    model = bench._update_launches(npad, nb, 4)
    m = npad - 4 * nb            # beyond the first group
    assert model[3][1] == 2 * m * m + 2 * m * 4 * nb
    m0, k = npad - nb, nb        # after panel 0: the next panel's column and row of tiles
    w = m0 - nb
    assert model[0][1] == 2 * m0 * nb + m0 * k + k * nb + 2 * nb * w + k * w
