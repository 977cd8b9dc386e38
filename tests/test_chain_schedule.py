"""Host-side check of the bulge-chain schedule of a multishift sweep (the
QR sweeps of the Schur factorisation; see csrc/schur.hip and k_chase in
csrc/hqr.hip).

A sweep over the active block of order N2 takes nb bulges (2 nb shifts) and
splits them into G chains, chain g holding cnb[g] bulges.  Bulge b of chain
g sits at position p = t - D[g] - 3b at sweep time t (its reflector acts on
rows/columns p..p+2 of the block; p = N2 - 2 is the 2x2 exit step), with
D[0] = 0 and D[g] = D[g-1] + adv + 3 cnb[g-1] + 1: chain g enters one window
width after the chain below it.  The sweep runs in phases of adv steps; in a
phase each chain with an active bulge owns the window
[max(0, pmin - 1), min(N2, pmax + 4)) of block rows and columns, pmin / pmax
the least / greatest active position.  The rules are restated here and
checked on random sweeps: the windows of a phase never overlap (so one
launch chases them side by side), every bulge visits every position once in
time order, and each step's rows (q-1 .. q+3, the bulge's column and the row
below its reflector) lie inside its window."""
import random

import pytest


def chains(nb, G):
    G = max(1, min(G, nb))
    cnb = [nb // G + (1 if g < nb % G else 0) for g in range(G)]
    return cnb


def schedule(N2, nb, G, adv):
    cnb = chains(nb, G)
    G = len(cnb)
    D = [0] * G
    for g in range(1, G):
        D[g] = D[g - 1] + adv + 3 * cnb[g - 1] + 1
    ttot = D[G - 1] + (N2 - 2) + 3 * (cnb[G - 1] - 1) + 1
    phases = []
    for t0 in range(0, ttot, adv):
        t1 = min(t0 + adv, ttot)
        wins = []
        for g in range(G):
            r0, r1 = t0 - D[g], t1 - D[g]
            pmin = max(0, r0 - 3 * (cnb[g] - 1))
            pmax = min(N2 - 2, r1 - 1)
            if pmax < pmin:
                continue
            wins.append((g, max(0, pmin - 1), min(N2, pmax + 4), r0, r1))
        phases.append(wins)
    return cnb, phases


@pytest.mark.parametrize("seed", range(5))
def test_chain_windows_disjoint_and_complete(seed):
    rs = random.Random(seed)
    for _ in range(120):
        N2 = rs.randint(8, 1500)
        adv = rs.choice([4, 8, 24, 40, 48, 64])
        nb = rs.randint(1, 44)
        G = rs.randint(1, 4)
        cnb, phases = schedule(N2, nb, G, adv)
        assert sum(cnb) == nb
        seen = {}
        for wins in phases:
            for a in range(len(wins)):
                for b in range(a + 1, len(wins)):
                    wa, wb = wins[a], wins[b]
                    assert wa[2] <= wb[1] or wb[2] <= wa[1], (N2, nb, G, adv, wa, wb)
            for g, ws, we, r0, r1 in wins:
                # the window a chase launch gets is at most adv + 3 cnb + 1 wide
                assert we - ws <= adv + 3 * cnb[g] + 1
                for t in range(r0, r1):
                    for b in range(cnb[g]):
                        p = t - 3 * b
                        if p < 0 or p > N2 - 2:
                            continue
                        q = p - ws                     # local row of the reflector
                        assert q >= (0 if p == 0 else 1)
                        assert min(p + 3, N2 - 1) - ws <= we - ws - 1
                        key = (g, b, p)
                        assert key not in seen
                        seen[key] = t
        for g in range(len(cnb)):
            for b in range(cnb[g]):
                ts = [seen[(g, b, p)] for p in range(N2 - 1)]
                assert ts == sorted(ts) and len(set(ts)) == len(ts)
                # bulge b trails bulge b-1 by three positions at every time
                if b > 0:
                    assert all(seen[(g, b, p)] == seen[(g, b - 1, p)] + 3 for p in range(N2 - 1))


def test_single_chain_is_the_tight_sweep():
    """One chain reproduces the usual sweep: every bulge three rows behind
    the previous one, windows of adv steps and no gaps."""
    cnb, phases = schedule(300, 20, 1, 48)
    assert cnb == [20]
    assert all(len(w) <= 1 for w in phases)
    ttot = (300 - 2) + 3 * 19 + 1
    assert len(phases) == (ttot + 47) // 48
