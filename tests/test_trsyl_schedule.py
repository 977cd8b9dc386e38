"""Host-side check of the right-looking tile schedule of the GPU tri-solve
(the substitution step of Sec. 2.2.1 over tiles; see csrc/trsyl.hip).

Tile (I, J) of the nI x nJ tile grid lies on anti-diagonal d(I, J) =
nI-1-I+J and needs, before it is solved, the contributions of every tile
below it in its block column, (K, J) with K > I, and of every tile left of
it in its block row, (I, L) with L < J.  After anti-diagonal d is solved the
update kernel gives tile (I, J) with d(I, J) > d the contributions of
(K, J), K = nI-1-d+J, and of (I, L), L = d-(nI-1-I), when those indices are
in range; in the mirrored (symmetric Lyapunov) mode tiles with 2J > d(I, J)
are never solved directly and receive nothing.  The rules are restated here
and checked for exact once-coverage, in the right order."""
import random

import pytest


def schedule(nI, nJ, mirror):
    got = {}
    for d in range(nI + nJ - 1):
        for I in range(nI):
            for J in range(nJ):
                dij = nI - 1 - I + J
                if dij <= d or (mirror and 2 * J > dij):
                    continue
                K, L = nI - 1 - d + J, d - (nI - 1 - I)
                if K < nI:
                    got.setdefault((I, J), []).append(("col", K, d))
                if L >= 0:
                    got.setdefault((I, J), []).append(("row", L, d))
    return got


@pytest.mark.parametrize("seed", range(6))
def test_each_contribution_once_and_before_the_tile(seed):
    rs = random.Random(seed)
    for _ in range(40):
        nI, nJ = rs.randint(1, 12), rs.randint(1, 12)
        mirror = rs.random() < 0.3
        if mirror:
            nJ = nI
        got = schedule(nI, nJ, mirror)
        for I in range(nI):
            for J in range(nJ):
                dij = nI - 1 - I + J
                if mirror and 2 * J > dij:
                    assert (I, J) not in got
                    continue
                ups = got.get((I, J), [])
                want = sorted([("col", K) for K in range(I + 1, nI)] + [("row", L) for L in range(J)])
                assert sorted((k, s) for k, s, _ in ups) == want, (nI, nJ, I, J)
                for kind, src, d in ups:
                    # the source tile is solved on anti-diagonal d, before this one
                    ds = nI - 1 - src + J if kind == "col" else nI - 1 - I + src
                    assert ds == d < dij
