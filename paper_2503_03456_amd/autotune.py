"""Autotuners of the Schur factorisation's QR-phase parameters and of the
batched Lyapunov path.

Coordinate search over (aedw, chasew, chains, nw, nb, adv, nsmall, nibble) --
the wavefronts of the AED and bulge-chase kernels, the bulge chains chased
side by side, the aggressive early deflation window, bulges per multishift
sweep, rows per bulge-chain window phase, the full-window cutoff and the
sweep-skip threshold (see
``sylv_schur_tune`` in include/sylv.h) -- timing ``sylv_schur`` on a matrix
of the benchmark recipe (normal, Re(eig) in [0.5, 5], 30% complex pairs) drawn
with a seed the benchmark does not use.  Each candidate is checked for a valid
Schur form (backward error) before its time counts.

    python -m paper_2503_03456_amd.autotune --n 2048 --report tune.json

prints one line per candidate and the best tuple per precision, installed in
the running process (the library's compiled-in defaults are the values this
search selected on MI355X).

    python -m paper_2503_03456_amd.autotune --batched --count 4096 --report tune_b.json

searches the batched path's tunables (``sylv_batched_tune``: Hessenberg
kernel buckets, band-QR LDS buckets, refinement passes per captured graph)
on the 4096-equation Lyapunov batch (orders U{16..256}), timing whole
batches (median of ``reps``) and requiring every equation at the tolerance.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import sys
import time

import numpy as np
import torch

from . import lib, _check

PREC = {"fp32": 1, "fp64": 0}
GRID = {
    "fp32": dict(nw=[24, 32, 40, 48, 64, 80, 96, 128], nb=[8, 12, 16, 20, 24, 32, 40, 44], adv=[24, 32, 40, 48, 64],
                 nsmall=[64, 96, 128, 140], nibble=[14, 20, 30, 40, 50, 65], aedw=[4, 7], chasew=[8, 16],
                 chains=[1, 2, 3, 4]),
    "fp64": dict(nw=[24, 32, 40, 48, 64, 80, 96], nb=[8, 12, 16, 20, 24, 32], adv=[24, 32, 40, 48],
                 nsmall=[64, 80, 98], nibble=[14, 20, 30, 40, 50, 65], aedw=[4, 7], chasew=[8, 16],
                 chains=[1, 2, 3, 4]),
}
ORDER = ["chains", "aedw", "chasew", "nw", "nb", "adv", "nsmall", "nibble"]
KEYS = ["nsmall", "nw", "nb", "adv", "nibble", "aedw", "chasew", "chains"]


def get(prec):
    v = (ctypes.c_int * 8)()
    _check(lib().sylv_schur_tune_get(PREC[prec], v), "sylv_schur_tune_get")
    return dict(zip(KEYS, list(v)))


def set_(prec, t):
    return lib().sylv_schur_tune(PREC[prec], t["nsmall"], t["nw"], t["nb"], t["adv"], t["nibble"], t["aedw"],
                                 t["chasew"], t["chains"])


def _matrix(n, seed):
    import workloads
    A, _, _, _ = workloads.normal_coeff(seed, n, 0.5, 5.0)
    return A


def time_schur(A64, prec, reps=1):
    dt = torch.float32 if prec == "fp32" else torch.float64
    A = torch.from_numpy(np.asfortranarray(A64)).to(dt).t().contiguous().t().cuda()
    from . import schur
    best = None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        T, U, st = schur(A)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        best = el if best is None else min(best, el)
    Td, Ud = T.double().cpu().numpy(), U.double().cpu().numpy()
    res = np.linalg.norm(A64 - Ud @ Td @ Ud.T) / np.linalg.norm(A64)
    ok = st == 0 and res < (1e-4 if prec == "fp32" else 1e-12)
    return best, ok, res


def tune(n=2048, precs=("fp32", "fp64"), seed=7, reps=1, progress=True, rounds=1):
    A = _matrix(n, seed)
    out = {}
    for prec in precs:
        cur = get(prec)
        time_schur(A, prec)  # warm-up (workspace, code objects)
        base, ok, _ = time_schur(A, prec, reps)
        best_t = base
        hist = [dict(cur, seconds=base)]
        if progress:
            print(f"[tune {prec}] start {cur} {base:.3f} s", flush=True)
        for key in ORDER * rounds:
            for val in GRID[prec][key]:
                if val == cur[key]:
                    continue
                cand = dict(cur, **{key: val})
                if set_(prec, cand) != 0:
                    continue
                t, ok, res = time_schur(A, prec, reps)
                hist.append(dict(cand, seconds=t, ok=bool(ok)))
                if progress:
                    print(f"[tune {prec}] {key}={val} {t:.3f} s ok={ok} res={res:.1e}", flush=True)
                if ok and t < best_t:
                    best_t, cur = t, cand
            set_(prec, cur)
        out[prec] = {"best": cur, "seconds": best_t, "start_seconds": base, "n": n, "seed": seed,
                     "history": hist}
        if progress:
            print(f"[tune {prec}] best {cur} {best_t:.3f} s (start {base:.3f} s)", flush=True)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--rounds", type=int, default=2)
    ap.add_argument("--prec", default="fp32,fp64")
    ap.add_argument("--report", default=None)
    ap.add_argument("--batched", action="store_true", help="tune the batched Lyapunov path instead")
    ap.add_argument("--count", type=int, default=4096)
    a = ap.parse_args(argv)
    if a.batched:
        res = tune_batched(a.count, reps=max(a.reps, 3), rounds=a.rounds)
        print(json.dumps({k: v for k, v in res.items() if k != "history"}), flush=True)
        if a.report:
            with open(a.report, "w") as fh:
                json.dump(res, fh, indent=1)
        return
    res = tune(a.n, tuple(a.prec.split(",")), a.seed, a.reps, rounds=a.rounds)
    summ = {p: {k: v for k, v in r.items() if k != "history"} for p, r in res.items()}
    print(json.dumps(summ), flush=True)
    if a.report:
        with open(a.report, "w") as fh:
            json.dump(res, fh, indent=1)



BGRID = {
    "hess": [(128, 64), (112, 64), (96, 64), (128, 48), (96, 48), (64, 48), (128, 32)],
    "band": [(180, 128, 0), (200, 160, 128), (224, 180, 128), (192, 144, 96), (180, 0, 0), (160, 112, 0),
             (212, 168, 120), (200, 144, 0), (240, 200, 160)],
    "gpasses": [2, 3, 4],
}


def get_batched():
    v = (ctypes.c_int * 6)()
    _check(lib().sylv_batched_tune_get(v), "sylv_batched_tune_get")
    return {"hess": (v[0], v[1]), "band": (v[2], v[3], v[4]), "gpasses": v[5]}


def set_batched(t):
    return lib().sylv_batched_tune(t["hess"][0], t["hess"][1], t["band"][0], t["band"][1], t["band"][2],
                                   t["gpasses"])


def tune_batched(count=4096, reps=3, rounds=1, progress=True):
    import workloads
    from . import solve_batched, batched_workspace_size
    sizes = workloads.config4_sizes()[:count]

    def dev(a):
        return torch.from_numpy(np.asfortranarray(a)).t().contiguous().t().cuda()

    eqs = []
    for i, n in enumerate(sizes):
        A, C, _ = workloads.config4_item(i, int(n))
        eqs.append((dev(A), dev(C)))
    Xs = [torch.empty((int(n), int(n)), dtype=torch.float64, device="cuda").t() for n in sizes]
    work = torch.empty(batched_workspace_size([1] * count, list(sizes), list(sizes)), dtype=torch.uint8,
                       device="cuda")

    def run():
        solve_batched(eqs, Xs=Xs, work=work)
        torch.cuda.synchronize()
        times, ok = [], True
        for _ in range(reps):
            t0 = time.perf_counter()
            _, infos = solve_batched(eqs, Xs=Xs, work=work)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            ok = ok and all(i["rel_res"] <= 1e-14 for i in infos)
        return float(np.median(times)), ok

    cur = get_batched()
    base, _ = run()
    best_t, hist = base, [dict(cur, seconds=base)]
    if progress:
        print(f"[tune batched] start {cur} {base * 1e3:.1f} ms", flush=True)
    for key in ["hess", "band", "gpasses"] * rounds:
        for val in BGRID[key]:
            if val == cur[key]:
                continue
            cand = dict(cur, **{key: val})
            if set_batched(cand) != 0:
                continue
            t, ok = run()
            hist.append(dict(cand, seconds=t, ok=ok))
            if progress:
                print(f"[tune batched] {key}={val} {t * 1e3:.1f} ms ok={ok}", flush=True)
            if ok and t < best_t:
                best_t, cur = t, cand
        set_batched(cur)
    return {"best": cur, "seconds": best_t, "start_seconds": base, "count": count, "history": hist}


if __name__ == "__main__":
    main()
