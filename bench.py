"""Throughput benchmark: solves/s and TFLOP/s at binary64-level residual,
mixed precision (binary32 Schur + binary64 refinement) vs plain binary64
Bartels-Stewart, on one MI355X.

Workload (default): the 2048 x 2048 Sylvester equation with normal
coefficients A = Q_A D_A Q_A^T, B = Q_B D_B Q_B^T (Re(eig) ~ U[0.5, 5], 30% of
eigenvalues in complex pairs, Q Haar), C ~ N(0,1); seeds 2, 3, 4.  A "step"
is one full solve (both Schur forms, transforms, tri-solve, refinement to
relative residual <= 1e-14) through the C ABI with A, B, C resident in HBM.

Prints ONE JSON line.  Run `python bench.py --help` for options.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAKS = {  # MI355X published dense peaks
    "hbm_GBps": 8000.0, "fp64_TFLOPs": 78.6, "fp32_TFLOPs": 157.3, "bf16_TFLOPs": 2500.0,
}

# HBM bytes per launch of a kernel, from rocprofv3 FETCH_SIZE and WRITE_SIZE
# runs of the default workload, each scaled by what the counter reads for a
# device copy of known size (bench.py --workload copy): x2.0 for FETCH_SIZE,
# x1.0 for WRITE_SIZE.  Valid for the kernel version the counters were taken
# on (profiles/hbm_traffic_sylvester_2048.md, profiles/hbm_traffic_symmetric_2048.md);
# None once the kernel changes.
TRAFFIC_BYTES = {"k_chase": (116.1 + 105.0) * 1024, "k_jac_pairs": (588.4 + 468.8) * 1024}

KERNEL_IDS = {"gemm_kernel": 1, "k_hess_col": 2, "k_hess_gemv": 3, "k_aed": 4, "k_chase": 5,
              "k_trsyl_diag": 6, "k_find_ktop": 7, "k_cast": 8, "k_sumsq_partial": 9,
              "k_bhess": 10, "k_bschur": 11, "k_btrsyl": 12, "gemm_batched_kernel": 13,
              "k_jac_pairs": 14, "k_jac_apply": 15}


def bs_flops(m, n, lyap=False):
    """Bartels-Stewart flop count (paper Sec. 2.2.1): 25(m^3+n^3)+5mn(m+n); Lyapunov 35 n^3."""
    return 35.0 * n ** 3 if lyap else 25.0 * (m ** 3 + n ** 3) + 5.0 * m * n * (m + n)


def mixed_flops(m, n, k):
    """Executed flops of the mixed path with k corrections:
    low: 25(m^3+n^3) + 5(k+1) mn(m+n); binary64: 2(k+1) mn(m+n) (residuals)."""
    a, b = m ** 3 + n ** 3, m * n * (m + n)
    return 25.0 * a + 5.0 * (k + 1) * b, 2.0 * (k + 1) * b


def sym_flops(m, n):
    """Symmetric-coefficient route (paper Sec. 2.2.2): eigen-decompositions
    9(m^3+n^3), transforms and back-transform 4mn(m+n), elementwise solve."""
    return 9.0 * (m ** 3 + n ** 3) + 4.0 * m * n * (m + n) + 2.0 * m * n


def host_cpu():
    """Model name of the host CPU (from /proc/cpuinfo) and its logical core count."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count() or 1


def forward_error(np, cfg, X, workload):
    """||X - X*||_F / ||X*||_F against the closed-form block-diagonal route of
    the normal constructions (no Schur factorisation involved); None for
    workloads without one."""
    if "DA" not in cfg and "QA" not in cfg:
        return None
    Xh = X.detach().cpu().numpy()
    if workload == "sym":
        QA, QB, la, lb = cfg["QA"], cfg["QB"], cfg["eigA"], cfg["eigB"]
        Xe = QA @ ((QA.T @ cfg["C"] @ QB) / (la[:, None] + lb[None, :])) @ QB.T
    else:
        sys.path.insert(0, os.path.join(ROOT, "tests"))
        from exact_route import exact_solution
        Xe = exact_solution(cfg)
    return float(np.linalg.norm(Xh - Xe) / np.linalg.norm(Xe))


def kappa_est(np, cfg):
    lam = np.abs(np.asarray(cfg["eigA"])[:, None] + np.asarray(cfg["eigB"])[None, :])
    return float(lam.max() / lam.min())


def measure_rho(torch, sy, n=2048, reps=5):
    """rho = cost of a binary32 flop / cost of a binary64 flop on this chip,
    measured as the ratio of the library's own n^3 GEMM times (binary32 MFMA
    vs binary64 MFMA), with HIP events on the current stream."""
    out = {}
    for name, dt in (("fp32", torch.float32), ("fp64", torch.float64)):
        # column-major views (the library's layout, so the binding copies nothing)
        a = torch.randn(n, n, dtype=dt, device="cuda").t()
        b = torch.randn(n, n, dtype=dt, device="cuda").t()
        c = torch.empty(n, n, dtype=dt, device="cuda").t()
        sy.gemm(a, b, c)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            sy.gemm(a, b, c)
        e1.record()
        torch.cuda.synchronize()
        out[name] = e0.elapsed_time(e1) / reps
    return {"rho": out["fp32"] / out["fp64"], "gemm_ms": out, "gemm_n": n,
            "tflops": {k: 2.0 * n ** 3 / (v * 1e-3) / 1e12 for k, v in out.items()}}


def predicted_speedup(m, n, k, rho):
    """Flop-model speedup of the mixed path over plain binary64
    Bartels-Stewart: (25a + 5b) / (rho (25a + 5(k+1) b) + 2(k+1) b),
    a = m^3 + n^3, b = mn(m+n) (paper Sec. 2.2.1 and Sec. 5 cost terms)."""
    a, b = m ** 3 + n ** 3, m * n * (m + n)
    return (25.0 * a + 5.0 * b) / (rho * (25.0 * a + 5.0 * (k + 1) * b) + 2.0 * (k + 1) * b)


def scipy_context(np, sample_n, target_m, target_n):
    """scipy.linalg.solve_sylvester (LAPACK gees + trsyl on the installed
    BLAS) on the same recipe at a smaller size, scaled by the flop model; a
    library reference point, not a target."""
    try:
        import scipy.linalg as sl
    except ImportError:
        return None
    import workloads
    cfg = workloads.config2(m=sample_n, n=sample_n)
    t0 = time.perf_counter()
    Xs = sl.solve_sylvester(cfg["A"], cfg["B"], cfg["C"])
    dt = time.perf_counter() - t0
    r = cfg["C"] - cfg["A"] @ Xs - Xs @ cfg["B"]
    rr = np.linalg.norm(r) / (np.linalg.norm(cfg["C"]) + np.linalg.norm(Xs) *
                              (np.linalg.norm(cfg["A"]) + np.linalg.norm(cfg["B"])))
    scale = bs_flops(sample_n, sample_n) / bs_flops(target_m, target_n)
    threads = os.environ.get("OMP_NUM_THREADS") or str(os.cpu_count())
    return {"value": scale / dt, "unit": "solves/s", "threads": threads,
            "sample": (f"scipy.linalg.solve_sylvester at m=n={sample_n} ({dt:.2f} s, rel_res {rr:.1e}), "
                       f"scaled to m={target_m} n={target_n} by the 25(m^3+n^3)+5mn(m+n) flop model")}


def c4_block(np, torch, sy, count, reps):
    """Compact record of the batched Lyapunov workload (count equations of
    orders U{16..256}): batch time, solves/s, worst relative residual,
    fallbacks; the library's captured graph path (nothing armed)."""
    items, sizes = c4_batch(count)

    def dev(a):
        return torch.from_numpy(np.asfortranarray(a)).t().contiguous().t().cuda()

    eqs = [(dev(A), dev(C)) for A, C, _ in items]
    Xs = [torch.empty((int(n), int(n)), dtype=torch.float64, device="cuda").t() for n in sizes]
    kinds = [1] * len(items)
    work = torch.empty(sy.batched_workspace_size(kinds, list(sizes), list(sizes)), dtype=torch.uint8,
                       device="cuda")
    sy.solve_batched(eqs, Xs=Xs, work=work)
    torch.cuda.synchronize()
    per, infos = [], None
    for _ in range(reps):
        t0 = time.perf_counter()
        infos = sy.solve_batched(eqs, Xs=Xs, work=work)[1]
        torch.cuda.synchronize()
        per.append(time.perf_counter() - t0)
    dt = float(np.median(per))
    n3 = (sizes.astype(float) ** 3).sum()
    del eqs, Xs, work
    torch.cuda.empty_cache()
    return {"workload": f"batched lyapunov, {count} equations, n~U{{16..256}}", "batch_ms_median": dt * 1e3,
            "batch_ms_min": min(per) * 1e3, "solves_per_s": count / dt,
            "max_rel_res": max(i["rel_res"] for i in infos),
            "all_solves_at_tol": all(i["rel_res"] <= 1e-14 for i in infos),
            "iterations_max": int(max(i["iterations"] for i in infos)),
            "fell_back": int(sum(i["fell_back"] for i in infos)),
            "tflops_bs_equivalent": 35.0 * n3 / dt / 1e12}


def load_workload(name):
    import workloads
    if name == "sym":
        cfg = workloads.config_sym()
        return cfg, "sylvester m=n=2048, symmetric A,B (eig U[0.5,5]), C~N(0,1)"
    if name == "c2":
        cfg = workloads.config2()
        return cfg, "sylvester m=n=2048, normal A,B (Re eig U[0.5,5], 30% complex pairs), C~N(0,1)"
    if name.startswith("c3"):
        j = int(name[2:] or "0")
        cfg = workloads.config3(j)
        return cfg, f"sylvester m=4096 n=1024, sep(A,-B)=delta={cfg['delta']:.0e}"
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(sample_n, target_m, target_n):
    """Time the CPU oracle (plain C, binary64, one thread) on the same recipe
    at a smaller size and scale by the Bartels-Stewart flop model."""
    import oracle
    import workloads
    cfg = workloads.config2(m=sample_n, n=sample_n)
    t0 = time.perf_counter()
    X, st = oracle.bs_solve(cfg["A"], cfg["B"], cfg["C"])
    dt = time.perf_counter() - t0
    rr = oracle.rel_residual(cfg["A"], cfg["B"], cfg["C"], X)
    scale = bs_flops(sample_n, sample_n) / bs_flops(target_m, target_n)
    return {"value": (1.0 / dt) * scale, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "host_cpu": host_cpu()[0], "host_logical_cores": host_cpu()[1],
            "sample": (f"one oracle solve of the same recipe at m=n={sample_n} "
                       f"({dt:.2f} s, rel_res {rr:.1e}), scaled to m={target_m} n={target_n} "
                       f"by the 25(m^3+n^3)+5mn(m+n) flop model")}


def cpu_baseline_sym(sample_n, target_m, target_n):
    """Time the oracle's symmetric route (plain C cyclic Jacobi, binary64,
    one thread) on the same recipe at a smaller size, scaled by the
    Sec. 2.2.2 flop model."""
    import oracle
    import workloads
    cfg = workloads.config_sym(m=sample_n, n=sample_n)
    t0 = time.perf_counter()
    X = oracle.sym_solve(cfg["A"], cfg["B"], cfg["C"])
    dt = time.perf_counter() - t0
    rr = oracle.rel_residual(cfg["A"], cfg["B"], cfg["C"], X)
    scale = sym_flops(sample_n, sample_n) / sym_flops(target_m, target_n)
    return {"value": (1.0 / dt) * scale, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "host_cpu": host_cpu()[0], "host_logical_cores": host_cpu()[1],
            "sample": (f"one oracle symmetric-route solve of the same recipe at m=n={sample_n} "
                       f"({dt:.2f} s, rel_res {rr:.1e}), scaled to m={target_m} n={target_n} "
                       f"by the 9(m^3+n^3)+4mn(m+n) flop model")}


def c4_batch(count):
    import workloads
    sizes = workloads.config4_sizes()[:count]
    return [workloads.config4_item(i, int(n)) for i, n in enumerate(sizes)], sizes


def cpu_baseline_batched(items, sizes, sample):
    """The CPU oracle (plain C, binary64) on a sample of the batch, one
    equation per host thread, scaled to the whole batch by sum n^3."""
    import concurrent.futures as cf
    import oracle
    idx = list(range(0, len(items), max(1, len(items) // sample)))[:sample]
    cores = os.cpu_count() or 1
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=cores) as ex:
        list(ex.map(lambda i: oracle.lyap_solve(items[i][0], items[i][1]), idx))
    dt = time.perf_counter() - t0
    n3 = sizes.astype(float) ** 3
    scale = n3[idx].sum() / n3.sum()
    return {"value": len(items) * scale / dt, "unit": "solves/s", "cores": cores, "kind": "oracle",
            "host_cpu": host_cpu()[0],
            "sample": (f"{len(idx)} equations of the batch (every {max(1, len(items) // sample)}th) "
                       f"solved by the oracle on {cores} threads in {dt:.2f} s, scaled to the "
                       f"{len(items)}-equation batch by sum n^3")}


def main_batched(args, np, torch, sy):
    import ctypes
    items, sizes = c4_batch(args.count)
    desc = (f"batched lyapunov, {len(items)} equations, n~U{{16..256}} (sum n^3 = "
            f"{(sizes.astype(float) ** 3).sum():.3e}), stable normal A (Re eig U[-5,-0.1], 30% "
            "complex pairs), C=-BB^T with B n x 4")

    def dev(a):
        return torch.from_numpy(np.asfortranarray(a)).t().contiguous().t().cuda()

    eqs = [(dev(A), dev(C)) for A, C, _ in items]
    Xs = [torch.empty((int(n), int(n)), dtype=torch.float64, device="cuda").t() for n in sizes]
    kinds = [1] * len(items)
    work = torch.empty(sy.batched_workspace_size(kinds, list(sizes), list(sizes)), dtype=torch.uint8,
                       device="cuda")
    torch.cuda.synchronize()

    def run(**kw):
        return sy.solve_batched(eqs, Xs=Xs, work=work, **kw)[1]

    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    lib = sy.lib()
    batched_kernels = ("k_bhess", "k_bschur", "k_btrsyl", "gemm_batched_kernel")
    kname = args.roofline_kernel if args.roofline_kernel in batched_kernels else "k_bschur"
    lib.sylv_profile_end.argtypes = [ctypes.POINTER(ctypes.c_long), ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double)]
    # timed region: nothing armed, so the batch runs through its captured graph
    infos, per = None, []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s0 = time.perf_counter()
        infos = run()
        torch.cuda.synchronize()
        per.append(time.perf_counter() - s0)
    t1 = time.perf_counter()
    dt = (t1 - t0) / args.steps
    # roofline: separate batches with the kernel's launches bracketed by HIP
    # events (armed profiling switches the batch to eager launches)
    nl, tot, work_acc = ctypes.c_long(0), ctypes.c_double(0.0), ctypes.c_double(0.0)
    if args.roofline_steps > 0:
        lib.sylv_profile_begin(KERNEL_IDS[kname])
        for _ in range(args.roofline_steps):
            run()
        torch.cuda.synchronize()
        lib.sylv_profile_end(ctypes.byref(nl), ctypes.byref(tot), ctypes.byref(work_acc))
    ok = all(i["rel_res"] <= 1e-14 for i in infos)
    iters = [i["iterations"] for i in infos]
    n3 = (sizes.astype(float) ** 3).sum()
    kbar = float(np.mean(iters))
    # plain binary64 (single-equation path) on a sample, scaled by sum n^3
    t64 = None
    if args.fp64_steps > 0:
        idx = list(range(0, len(items), max(1, len(items) // 128)))[:128]
        sub = [eqs[i] for i in idx]
        sy.solve_batched(sub, low="fp64")
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        sy.solve_batched(sub, low="fp64")
        torch.cuda.synchronize()
        t64 = (time.perf_counter() - s0) * n3 / (sizes[idx].astype(float) ** 3).sum()
    roof = None
    if nl.value > 0:
        roof = roofline_entry(kname, nl.value, tot.value, work_acc.value, args.roofline_steps, dt)
        roof["note"] = "eager launches (profiling armed); the timed batches replay the captured graph"
    out = {
        "metric": "solves/s and TFLOP/s at FP64-level residual: mixed-precision vs plain FP64",
        "value": (len(items) / dt) if ok else 0.0,
        "unit": "solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": desc, "count": len(items), "path": "batched fp32 Schur + fp64 refinement",
                   "tol": 1e-14},
        "ms_median": 1e3 * float(np.median(per)), "ms_min": 1e3 * min(per),
        "rel_res": max(i["rel_res"] for i in infos), "all_solves_at_tol": ok,
        "iterations_mean": kbar, "iterations_max": int(max(iters)),
        "fell_back": int(sum(i["fell_back"] for i in infos)),
        "tflops_bs_equivalent": 35.0 * n3 / dt / 1e12,
        "tflops_executed": {"fp32": (25.0 + 10.0 * (kbar + 1)) * n3 / dt / 1e12,
                            "fp64": 4.0 * (kbar + 1) * n3 / dt / 1e12},
        "fp64_plain": None if t64 is None else {
            "solves_per_s": len(items) / t64, "ms_per_batch": t64 * 1e3,
            "note": "single-equation binary64 path on 128 sampled equations, scaled by sum n^3"},
        "speedup_vs_fp64": None if t64 is None else t64 / dt,
        "roofline": roof, "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_batched(items, sizes, args.cpu_sample_eqs)
    print(json.dumps(out), flush=True)


def sweep_c3(args, np, torch, sy):
    """Config 3 (m = 4096, n = 1024, sep = delta = 1e-1 .. 1e-6): one solve per
    delta and path (binary32 forms, BF16-update forms, plain binary64), with
    iterations, escalation, relative residual and the forward error against
    the exact block-diagonal solution of the normal construction."""
    import workloads
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from exact_route import exact_solution

    def dev(a):
        return torch.from_numpy(np.asfortranarray(a)).t().contiguous().t().cuda()

    from paper_2503_03456_amd import selector
    selector.install(*selector.load())   # the committed weights, for low = "auto"
    rows = []
    for j in range(args.c3_first, 6):
        cfg = workloads.config3(j)
        A, B, C = dev(cfg["A"]), dev(cfg["B"]), dev(cfg["C"])
        Xe = exact_solution(cfg)
        row = {"delta": cfg["delta"], "kappa_est": kappa_est(np, cfg),
               "forward_error_bound": 100 * 2.0 ** -53 * kappa_est(np, cfg)}
        for low in ("fp32", "bf16", "fp64", "auto"):
            sy.solve(A, B, C, low=low)   # warm
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            X, info = sy.solve(A, B, C, low=low)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            fe = float(np.linalg.norm(X.cpu().numpy() - Xe) / np.linalg.norm(Xe))
            row[low] = {"seconds": dt, "iterations": info["iterations"], "fell_back": info["fell_back"],
                        "precision_used": info["precision_used"], "rel_res": info["rel_res"],
                        "forward_error": fe, "sep_est": info["sep_est"], "chosen": info["chosen"]}
        rows.append(row)
        print(f"[c3] delta={cfg['delta']:.0e} " + " ".join(
            f"{k}:{row[k]['seconds']:.2f}s/it{row[k]['iterations']}/fb{row[k]['fell_back']}"
            for k in ("fp32", "bf16", "fp64", "auto")), file=sys.stderr, flush=True)
    print(json.dumps({"workload": "config 3 sweep, sylvester m=4096 n=1024", "rows": rows}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--fp64-steps", type=int, default=2, help="timed plain binary64 solves")
    ap.add_argument("--roofline-kernel", default="k_chase")
    ap.add_argument("--roofline-steps", type=int, default=2,
                    help="solves (batches) run after the timed region with the roofline kernel's "
                         "launches bracketed by HIP events")
    ap.add_argument("--rho", type=int, default=1, help="measure rho (binary32/binary64 GEMM time ratio)")
    ap.add_argument("--c4-count", type=int, default=4096,
                    help="default workload: equations of the batched Lyapunov block added to the line (0: off)")
    ap.add_argument("--c4-reps", type=int, default=3)
    ap.add_argument("--scipy-n", type=int, default=1024,
                    help="size of the scipy.linalg.solve_sylvester context sample (0: off)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-n", type=int, default=768)
    ap.add_argument("--count", type=int, default=4096, help="equations of the batched workload (c4)")
    ap.add_argument("--cpu-sample-eqs", type=int, default=1024)
    ap.add_argument("--c3-first", type=int, default=0, help="first delta index of the c3sweep workload")
    ap.add_argument("--alg", default="orig", choices=["orig", "orth", "inv", "sym"],
                    help="mixed path: refinement in the original basis (orig), the paper's Alg. 4.1 (orth) "
                         "or Alg. 4.2 (inv); the sym workload always runs the symmetric-coefficient "
                         "route (sym), with the plain binary64 symmetric route as its baseline")
    ap.add_argument("--general-steps", type=int, default=1,
                    help="sym workload: timed solves of the same equation by the general path (context)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}): this solver has no "
              "multi-GPU path; the batched workload shards by equation across GPUs and the "
              "single solve would exchange Schur factors, neither is built here.", file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))

    import numpy as np
    import torch
    import paper_2503_03456_amd as sy

    if args.workload == "c4":
        return main_batched(args, np, torch, sy)
    if args.workload == "c3sweep":
        return sweep_c3(args, np, torch, sy)
    if args.workload == "copy":
        # calibration for hardware byte counters: device-to-device copies of a
        # known size (read 256 MiB + write 256 MiB per copy)
        a = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(args.steps):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"workload": "copy", "bytes_read_per_copy": a.numel() * 4,
                          "bytes_written_per_copy": a.numel() * 4, "copies": args.steps}), flush=True)
        return
    cfg, desc = load_workload(args.workload)
    m, n = cfg["C"].shape
    if args.workload == "sym":
        args.alg = "sym"
        if args.roofline_kernel == "k_chase":
            args.roofline_kernel = "k_jac_pairs"

    def dev(a):
        return torch.from_numpy(np.asfortranarray(a)).t().contiguous().t().cuda()

    A, B, C = dev(cfg["A"]), dev(cfg["B"]), dev(cfg["C"])
    X = torch.empty((n, m), dtype=torch.float64, device="cuda").t()
    work = torch.empty(max(sy.workspace_size(m, n, low="fp32", alg=args.alg), sy.workspace_size(m, n, low="fp64")),
                       dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()

    def run(low, alg=None):
        if alg is None:
            alg = args.alg if (low != "fp64" or args.alg == "sym") else "orig"
        return sy.solve(A, B, C, X=X, work=work, low=low, alg=alg)[1]

    for _ in range(args.warmup):
        run("fp32")
    if args.fp64_steps > 0:
        run("fp64")
    torch.cuda.synchronize()

    # timed region: K mixed-precision solves, nothing armed (no per-launch
    # events, no profiling hooks); each solve is synchronous, so per-solve
    # wall times give the median and the minimum
    infos, per = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s0 = time.perf_counter()
        infos.append(run("fp32"))
        per.append(time.perf_counter() - s0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dt = (t1 - t0) / args.steps
    ok = all(i["rel_res"] <= 1e-14 for i in infos)
    iters = infos[-1]["iterations"]
    fwd = forward_error(np, cfg, X, args.workload)

    # plain binary64 path (the comparison, not the headline value)
    t64 = None
    inf64 = None
    per64 = []
    if args.fp64_steps > 0:
        torch.cuda.synchronize()
        for _ in range(args.fp64_steps):
            s0 = time.perf_counter()
            inf64 = run("fp64")
            per64.append(time.perf_counter() - s0)
        torch.cuda.synchronize()
        t64 = sum(per64) / len(per64)
        fwd64 = forward_error(np, cfg, X, args.workload)

    # symmetric workload: the general path on the same equation (context)
    tgen = None
    if args.alg == "sym" and args.general_steps > 0:
        run("fp32", alg="orig")
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        for _ in range(args.general_steps):
            infg = run("fp32", alg="orig")
        torch.cuda.synchronize()
        tgen = (time.perf_counter() - s0) / args.general_steps

    # roofline of the dominant kernel: separate solves with that kernel's
    # launches bracketed by HIP events on their launch stream
    lib = sy.lib()
    kid = KERNEL_IDS[args.roofline_kernel]
    import ctypes
    lib.sylv_profile_end.argtypes = [ctypes.POINTER(ctypes.c_long), ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double)]
    nl, tot, work_acc = ctypes.c_long(0), ctypes.c_double(0.0), ctypes.c_double(0.0)
    if args.roofline_steps > 0:
        lib.sylv_profile_begin(kid)
        for _ in range(args.roofline_steps):
            run("fp32")
        torch.cuda.synchronize()
        lib.sylv_profile_end(ctypes.byref(nl), ctypes.byref(tot), ctypes.byref(work_acc))

    lo, hi = mixed_flops(m, n, iters)
    bsf = bs_flops(m, n)
    roof = None
    if nl.value > 0:
        roof = roofline_entry(args.roofline_kernel, nl.value, tot.value, work_acc.value,
                              args.roofline_steps, dt)
    out = {
        "metric": "solves/s and TFLOP/s at FP64-level residual: mixed-precision vs plain FP64",
        "value": (1.0 / dt) if ok else 0.0,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": desc, "m": m, "n": n,
                   "path": {"orig": "fp32 Schur + fp64 refinement",
                            "orth": "Alg. 4.1: fp32 Schur, fp64-orthonormalised factors, triangular-basis refinement",
                            "inv": "Alg. 4.2: fp32 Schur, fp64 inverses of the factors, triangular-basis refinement",
                            "sym": "symmetric route: fp32 block-Jacobi eigen-decompositions, elementwise solve, "
                                   "fp64 refinement"}[args.alg],
                   "tol": 1e-14},
        "ms_median": 1e3 * float(np.median(per)), "ms_min": 1e3 * min(per),
        "rel_res": max(i["rel_res"] for i in infos),
        "forward_error": fwd,
        "all_solves_at_tol": ok,
        "iterations": iters,
        "fell_back": infos[-1]["fell_back"],
        "tflops_bs_equivalent": bsf / dt / 1e12,
        "tflops_executed": {"fp32": lo / dt / 1e12, "fp64": hi / dt / 1e12},
        "fp64_plain": None if t64 is None else {
            "solves_per_s": 1.0 / t64, "ms_per_solve": t64 * 1e3, "ms_median": 1e3 * float(np.median(per64)),
            "ms_min": 1e3 * min(per64), "rel_res": inf64["rel_res"], "forward_error": fwd64,
            "tflops_bs_equivalent": bsf / t64 / 1e12},
        "speedup_vs_fp64": None if t64 is None else t64 / dt,
        "general_path": None if tgen is None else {
            "ms_per_solve": tgen * 1e3, "rel_res": infg["rel_res"],
            "note": "fp32 Schur + fp64 refinement on the same symmetric equation"},
        "roofline": roof,
        "cpu_baseline": None,
    }
    if args.alg == "sym":
        out["tflops_bs_equivalent"] = sym_flops(m, n) / dt / 1e12
        out["tflops_executed"] = None
        if out["fp64_plain"] is not None:
            out["fp64_plain"]["tflops_bs_equivalent"] = sym_flops(m, n) / t64 / 1e12
            out["fp64_plain"]["path"] = "plain binary64 symmetric route (block Jacobi, elementwise solve)"
    if "eigA" in cfg and "eigB" in cfg:
        kap = kappa_est(np, cfg)
        out["kappa_est"] = kap
        out["forward_error_bound"] = 100 * 2.0 ** -53 * kap
    if args.alg != "sym" and t64 is not None and args.rho:
        r = measure_rho(torch, sy)
        r["predicted_speedup"] = predicted_speedup(m, n, iters, r["rho"])
        r["measured_speedup"] = t64 / dt
        out["flop_model"] = r
    if args.c4_count > 0 and args.workload == "c2":
        out["batched_c4"] = c4_block(np, torch, sy, args.c4_count, args.c4_reps)
    if rank == 0 and not args.no_cpu_baseline:
        out["cpu_baseline"] = (cpu_baseline_sym(min(args.cpu_sample_n, 256), m, n) if args.alg == "sym"
                               else cpu_baseline(args.cpu_sample_n, m, n))
        if args.alg != "sym" and args.scipy_n > 0:
            out["scipy_context"] = scipy_context(np, args.scipy_n, m, n)
    if rank == 0:
        print(json.dumps(out), flush=True)


def roofline_entry(kname, launches, total_ms, work, steps, step_s):
    """Roofline object of the dominant kernel.  `work` is the algorithmic
    flop count the library accounted for the timed launches (k_aed, k_chase:
    every application of a 3x3 bulge reflector to a window row or column,
    including the accumulated orthogonal factor, 12 flops; gemm_kernel: 2mnk).
    The QR kernels work on an LDS-resident window with vector ALU arithmetic,
    so their roof is the fp32 vector peak of the chip."""
    avg_ms = total_ms / launches
    ach = work / (total_ms * 1e-3) / 1e12 if total_ms > 0 else 0.0
    bound = "alu" if kname in ("k_chase", "k_aed", "k_bschur", "k_bhess", "k_jac_pairs") else "mfma"
    peak = PEAKS["fp32_TFLOPs"]
    tb = TRAFFIC_BYTES.get(kname)
    return {"kernel": kname, "bound": bound, "achieved": ach, "peak": peak, "unit": "TFLOP/s",
            "frac": ach / peak, "traffic": tb, "avg_launch_ms": avg_ms,
            "launches_per_step": launches / steps, "work_per_launch_flops": work / launches,
            "share_of_step": (total_ms * 1e-3 / steps) / step_s}


if __name__ == "__main__":
    main()
