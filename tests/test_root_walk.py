"""The persistent final-step kernel's tile walk, emulated on the CPU: for
every grid of workgroups (a multiple of 8, also larger than the tile count,
as the shared launch of many reconstructions uses it) and every tile grid of
2^lgtm x 2^lgtn tiles, each tile is visited exactly once and every index
stays in range.  The formulas are those of the kernel: workgroup b serves
XCD b mod 8, slot b div 8; XCD x owns the contiguous range
[x * ceil(T/8), min((x+1) * ceil(T/8), T)); inside it the slots take every
nslots-th position; positions walk groups of 2^min(lgtm, 3) tile rows column
by column."""
import pytest


def visits(G, lgtm, lgtn):
    ntiles = 1 << (lgtm + lgtn)
    seen = []
    for b in range(G):
        xcd, slot = b & 7, b >> 3
        nslots = (G - xcd + 7) >> 3
        per = (ntiles + 7) >> 3
        r0 = xcd * per
        r1 = min(r0 + per, ntiles)
        mine = (r1 - r0 - slot + nslots - 1) // nslots if r1 > r0 + slot else 0
        lgm = min(lgtm, 3)
        for i in range(mine):
            idx = r0 + slot + i * nslots
            assert idx < ntiles
            grp, r = idx >> (lgm + lgtn), idx & ((1 << (lgm + lgtn)) - 1)
            tm, tn = (grp << lgm) | (r & ((1 << lgm) - 1)), r >> lgm
            assert tm < (1 << lgtm) and tn < (1 << lgtn)
            seen.append((tm << lgtn) | tn)
    return ntiles, seen


@pytest.mark.parametrize("G", [8, 16, 64, 256, 512])
def test_every_tile_once(G):
    for lgtm in range(0, 9):
        for lgtn in range(0, 9):
            ntiles, seen = visits(G, lgtm, lgtn)
            assert sorted(seen) == list(range(ntiles)), (G, lgtm, lgtn)
