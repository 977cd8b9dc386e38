"""Host-side check of the large-tile GEMM's workgroup-to-tile order
(gemm128_kernel in csrc/gemm.hip).

The hardware deals a launch's workgroups to the 8 XCDs round-robin
(workgroup b to XCD b mod 8).  When the tile count is a multiple of 8 the
kernel renumbers b so that XCD x takes the consecutive run
[x nblk/8, (x+1) nblk/8) of the order below; the order walks the tile grid in
groups of G = 4 tile rows, column by column inside a group (a last group of
fewer rows when tiles_m is not a multiple of 4).  The rules are restated here
and checked: every grid maps one to one onto its tiles; at 16 x 16 tiles
(2048^2 outputs) each XCD gets a 4 x 8 block, so its L2 streams 4 row panels
of op(A) and 8 column panels of op(B) instead of all 16 row panels; and on
larger grids the tiles an XCD holds at once (one per CU) span fewer panels
than whole tile columns would."""
import pytest

G = 4


def tile_of(b, tiles_m, tiles_n):
    nblk = tiles_m * tiles_n
    bid = b
    if nblk % 8 == 0:
        bid = (bid & 7) * (nblk >> 3) + (bid >> 3)
    per = G * tiles_n
    grp = bid // per
    m0 = grp * G
    gs = min(G, tiles_m - m0)
    r = bid - grp * per
    return m0 + r % gs, r // gs


@pytest.mark.parametrize("tiles_m", range(1, 41))
def test_order_is_a_bijection(tiles_m):
    for tiles_n in range(1, 41):
        got = [tile_of(b, tiles_m, tiles_n) for b in range(tiles_m * tiles_n)]
        assert sorted(got) == [(i, j) for i in range(tiles_m) for j in range(tiles_n)], (tiles_m, tiles_n)


def resident_panels(order, tiles_m, tiles_n, resident=32):
    """Panels (distinct tile rows + tile columns) each XCD streams while a
    chunk of `resident` consecutive tiles of its run (one per CU) is in
    flight, keyed by (XCD, chunk)."""
    nblk = tiles_m * tiles_n
    out = {}
    for b in range(nblk):
        tm, tn = order(b, tiles_m, tiles_n)
        rows, cols = out.setdefault((b % 8, (b >> 3) // resident), (set(), set()))
        rows.add(tm)
        cols.add(tn)
    return {k: (len(r), len(c)) for k, (r, c) in out.items()}


def column_major(b, tiles_m, tiles_n):
    """The order without row groups: each XCD's run walks whole tile columns."""
    nblk = tiles_m * tiles_n
    bid = (b & 7) * (nblk >> 3) + (b >> 3) if nblk % 8 == 0 else b
    return bid % tiles_m, bid // tiles_m


def test_square_2048_gives_each_xcd_a_4x8_block():
    assert resident_panels(tile_of, 16, 16) == {(x, 0): (4, 8) for x in range(8)}


@pytest.mark.parametrize("tiles_m,tiles_n", [(16, 16), (32, 8), (8, 16), (32, 32), (24, 16), (64, 64)])
def test_fewer_resident_panels_than_whole_columns(tiles_m, tiles_n):
    """While one tile per CU is resident, an XCD streams no more panels of
    op(A) and op(B) than with whole tile columns, and fewer in total on
    grids taller than 4 tile rows."""
    g = resident_panels(tile_of, tiles_m, tiles_n)
    p = resident_panels(column_major, tiles_m, tiles_n)
    assert g.keys() == p.keys()
    tot_g = sum(r + c for r, c in g.values())
    tot_p = sum(r + c for r, c in p.values())
    assert all(sum(g[k]) <= sum(p[k]) for k in g), (g, p)
    if tiles_m > G:
        assert tot_g < tot_p, (tot_g, tot_p)
