"""The placement rule both spreads use for a run of W = 4 taps (Eq. 1-2,
Eq. 7-8: the Projection Core on a periodic grid), checked on the host for
every tile extent the library can pick.

A spread workgroup owns a tile [lo, lo + TS) of an axis of G cells and
places a tap run starting at cell b (mod G) at the offset o = b - lo folded
into (-G/2, G/2]; taps o .. o + 3 that fall in [0, TS) are accumulated.  This
finds exactly the in-tile taps when TS <= G/2 (the library caps every spread
tile extent at the largest power of two not above G/2).  The second test
shows the failure the cap prevents: a 16-wide tile on an axis of 16 cells
loses the taps of runs that start past the middle."""
import pytest


def spread_extent(want: int, G: int) -> int:
    cap = 1
    while 2 * cap <= G // 2:
        cap *= 2
    return min(want, cap)


def folded_hits(b, lo, TS, G):
    o = (b - lo) % G
    if o > G // 2:
        o -= G
    if o < -(G // 2):
        o += G
    return sorted(o + t for t in range(4) if 0 <= o + t < TS)


def true_hits(b, lo, TS, G):
    cells = [(b + t) % G for t in range(4)]
    return sorted(c - lo for c in cells if lo <= c < lo + TS)


@pytest.mark.parametrize("G", list(range(16, 130, 2)))
@pytest.mark.parametrize("want", [4, 8, 16])
def test_capped_tiles_find_every_tap(G, want):
    TS = spread_extent(want, G)
    assert 4 <= TS <= G // 2
    for lo in range(0, G, TS):
        ext = min(TS, G - lo)  # the last tile of a ragged axis
        for b in range(G):
            assert folded_hits(b, lo, ext, G) == true_hits(b, lo, ext, G), (G, TS, lo, b)


def test_uncapped_tile_loses_taps():
    G, TS, lo = 16, 16, 0
    bad = [b for b in range(G) if folded_hits(b, lo, TS, G) != true_hits(b, lo, TS, G)]
    assert 10 in bad  # taps 10..13 lie in the tile but the fold puts the run at -6..-3
