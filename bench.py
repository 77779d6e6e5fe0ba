#!/usr/bin/env python3
"""Benchmark of the ChebFD polynomial filter on one MI355X.

One step = one full filter application (Alg. 1 on every block, Alg. 2 over the
blocks) to an n_s-vector search block of the Topi-64-64-32 lattice Hamiltonian
(n = 524288, 13 non-zeros per row, disorder W = 1, complex double,
SELL-32-256), n_s = 256 in blocks of n_b = 32, filter degree n_p = 1000.
Inputs are synthetic and resident in HBM before the timed region.

Prints one JSON line: the filter's algorithmic HBM bandwidth (the paper's
minimum-traffic model, Sect. 3.4) as `value`, the roofline of the fused step
kernel (its launches timed on their own), the same filter with c64 block
vectors (`filter_mixed`), the time to converged Ritz pairs of the whole
iteration in FP64, in mixed precision and in mixed precision with the learned
(n_p, n_s) on the same matrix, and the FP64 CPU oracle timed on a bounded
sample of the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E, published
METRIC = "Cheb filter HBM GB/s (% of peak); time to converged pairs, plain vs mixed"


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--lattice", type=str, default="64x64x32")
    ap.add_argument("--W", type=float, default=1.0)
    ap.add_argument("--n_s", type=int, default=256)
    ap.add_argument("--n_b", type=int, default=32)
    ap.add_argument("--n_p", type=int, default=1000)
    ap.add_argument("--prec", type=int, default=0, help="0 = FP64, 1 = mixed (c64 storage)")
    ap.add_argument("--cpu-baseline-seconds", type=float, default=15.0,
                    help="target CPU time of the oracle sample (0 disables)")
    ap.add_argument("--no-solve", action="store_true", help="skip the time-to-converged leg")
    ap.add_argument("--no-mixed-filter", action="store_true",
                    help="skip the c64 filter leg (timed after the FP64 filter when --prec 0)")
    ap.add_argument("--solve-prec", choices=("both", "fp64", "mixed"), default="both",
                    help="precisions of the time-to-converged leg")
    ap.add_argument("--solve-count", type=float, default=100.0,
                    help="eigenvalue count the symmetric search interval is sized for")
    ap.add_argument("--op-launches", type=int, default=200, help="launches of the fused step timed alone")
    ap.add_argument("--order", choices=("lattice", "natural"), default="lattice",
                    help="row order at ingest: lattice boxes/slabs (one box per XCD) or the natural order")
    return ap.parse_args()


# fused-step kernels (chebfd_step_kernel kinds): short name, source file
STEP_KERNELS = {0: ("cheb_lds", "filter_lds.hip"), 1: ("cheb_row", "filter_rows.hip"),
                2: ("cheb_multirow", "filter.hip"), 3: ("cheb_win", "filter_win.hip")}


def kernel_source_hash(kind: int) -> str:
    """Hash of the step kernel's source and the pack header it includes."""
    h = hashlib.sha256()
    for name in (STEP_KERNELS[kind][1], "step_io.h"):
        with open(os.path.join(HERE, "paper_1803_02156_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def counter_traffic(kind: int, prec: int, n_b: int, lattice: str, order: str):
    """HBM bytes per fused-step launch from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary, if it was taken on the current kernel source; else None."""
    name = (f"traffic_{STEP_KERNELS[kind][0]}_step_topi{lattice.replace('x', '-')}_"
            f"{'fp64' if prec == 0 else 'mixed'}_nb{n_b}_{order}.json")
    path = os.path.join(HERE, "profiles", name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_source_sha256_16") != kernel_source_hash(kind):
        return None
    return t["hbm_bytes_per_launch"]


def mixed_filter_leg(P, H, order, lattice, order_name, n_s, n_b, n_p, steps):
    """The same full filter with c64 block vectors and a c64 matrix (the mixed
    precision's filter stage): algorithmic GB/s, the fused step's average launch
    and the step kernel with its committed HBM traffic."""
    import torch
    from paper_1803_02156_amd import traffic
    from topi import random_phase_block
    n, nnz = len(H[0]) - 1, len(H[1])
    M = P.chebfd_matrix_build(*H, C=32, sigma=256, prec=1, order=order)
    lo, hi = P.chebfd_bounds(M)
    al, be, gam = P.chebfd_coefficients(lo, hi, -0.1, 0.1, n_p)
    X0 = random_phase_block(n, n_s, 45)
    x0 = torch.empty((n_s, n), dtype=torch.complex128, device="cuda")
    x0.copy_(torch.from_numpy(np.ascontiguousarray(X0.T)))
    del X0
    xb0 = P.chebfd_pack(M, x0.T, n_b)
    del x0
    xy = torch.empty_like(xb0)
    work = P.FilterWork(M, n_b, n_p, n_s, moments=True)
    stream = torch.cuda.current_stream()

    def step():
        xy.copy_(xb0)
        P.chebfd_filter(M, al, be, gam, n_s, n_b, xy, work=work)
    step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    gbs = traffic.filter_bytes(n, nnz, n_s, n_b, n_p, 1) / (ms * 1e-3) / 1e9
    avg_launch_s = ms * 1e-3 / ((n_s // n_b) * n_p)
    r, w = traffic.step_bytes(n, nnz, n_b, 1)
    kind = P.chebfd_step_kernel(M, n_b)
    out = {"value": round(gbs, 2), "unit": "GB/s", "ms_per_filter": round(ms, 3),
           "pct_of_hbm_peak": round(100.0 * gbs / HBM_PEAK_GBS, 2),
           "kernel": f"{STEP_KERNELS[kind][0]}_kernel<float,{n_b},kModeStep>",
           "avg_launch_us": round(avg_launch_s * 1e6, 3), "bytes_per_launch": r + w,
           "frac": round((r + w) / avg_launch_s / 1e9 / HBM_PEAK_GBS, 4),
           "traffic": counter_traffic(kind, 1, n_b, lattice, order_name),
           "kernel_source_sha256_16": kernel_source_hash(kind)}
    del xy, xb0, work, M
    torch.cuda.empty_cache()
    return out


def interval_for_count(P, M, target, seed=7, n_steps=1024, R=16):
    """Half width delta of the symmetric interval [-delta, delta] whose KPM count
    estimate (2 n_steps moments of R random-phase vectors, Jackson-damped window)
    is closest to `target`: the moments once on the device, the bisection on them."""
    lo_b, hi_b = P.chebfd_bounds(M)
    al, be, _ = P.chebfd_coefficients(lo_b, hi_b, -1e-3, 1e-3, 1)
    mu = P.chebfd_kpm_moments(M, al, be, n_steps, R, seed)

    def count(d):
        _, _, gc = P.chebfd_coefficients(lo_b, hi_b, -d, d, 2 * n_steps - 1)
        return float(M.n * np.dot(gc, mu))
    half = max(abs(lo_b), abs(hi_b))
    a, b = 1e-4 * half, 0.5 * half
    for _ in range(60):
        mid = 0.5 * (a + b)
        if count(mid) < target:
            a = mid
        else:
            b = mid
        if b - a < 1e-6 * b:
            break
    return 0.5 * (a + b), count(0.5 * (a + b))


def time_to_converged(P, H, Nx, Ny, Nz, W, n_s, n_b, n_p, target, order, which="both"):
    """Full ChebFD runs (filter, SVQB, Rayleigh-Ritz, residuals, restarts) in FP64 and
    mixed precision on the same matrix and interval; wall time from the first launch
    to the synchronised end, matrix build excluded."""
    import torch
    M64 = P.chebfd_matrix_build(*H, prec=0, order=order)
    delta, cnt = interval_for_count(P, M64, target)
    out = {"workload": f"Topi-{Nx}-{Ny}-{Nz} (W={W}), interval [-{delta:.6g}, {delta:.6g}] "
                       f"(KPM count estimate {cnt:.1f}, 2048 moments), n_s={n_s}, n_b={n_b}, n_p={n_p}",
           "interval": [-delta, delta], "count_est_kpm": cnt}
    runs = {}
    for name, prec in (("fp64", 0), ("mixed", 1)):
        if which not in ("both", name):
            continue
        M = M64 if prec == 0 else P.chebfd_matrix_build(*H, prec=1, order=order)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = P.chebfd_solve(M, M64, -delta, delta, n_s, n_p, n_b, seed=43, max_iter=12, want_vectors=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        nf = r.n_found
        runs[name] = r
        st = r.stats
        out[name] = {
            "seconds": round(dt, 3), "status": r.status, "iterations": st.iterations, "n_found": nf,
            "max_resid": float(np.max(r.resid[:nf])) if nf else None,
            "tol": 1e-9 if prec == 0 else 1e-7,
            "t_filter": round(st.t_filter, 3), "t_orth": round(st.t_orth, 3), "t_rr": round(st.t_rr, 3),
            "t_resid": round(st.t_resid, 3),
            "filter_gbs": round(st.filter_bytes / st.t_filter / 1e9, 1) if st.t_filter > 0 else None,
        }
        print(f"# solve {name}: {dt:.2f} s, status {r.status}, {st.iterations} iterations, "
              f"{nf} pairs", file=sys.stderr, flush=True)
        del M
    if which == "both":
        # mixed precision with the trained predictor's (n_p, n_s) for this matrix and interval
        from paper_1803_02156_amd import predictor as PR
        if os.path.exists(PR.DEFAULT_WEIGHTS):
            pred = PR.load(PR.DEFAULT_WEIGHTS)
            f, cnt, _, _ = P.chebfd_features(M64, -delta, delta, 7)
            lp, ls = PR.choose(pred, f, cnt, pred["kappa"])
            ls = max(n_b, ls // n_b * n_b)
            M = P.chebfd_matrix_build(*H, prec=1, order=order)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = P.chebfd_solve(M, M64, -delta, delta, ls, lp, n_b, seed=43, max_iter=12, want_vectors=False)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            nf = r.n_found
            out["mixed_learned"] = {"seconds": round(dt, 3), "status": r.status, "iterations": r.stats.iterations,
                                    "n_found": nf, "n_p": lp, "n_s": ls,
                                    "max_resid": float(np.max(r.resid[:nf])) if nf else None}
            print(f"# solve mixed + learned (n_p {lp}, n_s {ls}): {dt:.2f} s, status {r.status}, "
                  f"{r.stats.iterations} iterations, {nf} pairs", file=sys.stderr, flush=True)
            del M
    if len(runs) == 2:
        a, b = runs["fp64"], runs["mixed"]
        if a.n_found == b.n_found and a.n_found > 0:
            out["mixed"]["max_abs_dtheta_vs_fp64"] = float(np.max(np.abs(np.sort(a.theta[:a.n_found]) -
                                                                          np.sort(b.theta[:b.n_found]))))
        out["speedup_mixed_vs_fp64"] = round(out["fp64"]["seconds"] / out["mixed"]["seconds"], 3)
        ml = out.get("mixed_learned")
        if ml is not None:
            ok = ml["status"] == 0 and ml["n_found"] >= a.n_found
            ml["converged_all_pairs"] = ok
            # a speedup only for a run that found every pair the FP64 run found
            out["speedup_mixed_learned_vs_fp64"] = round(out["fp64"]["seconds"] / ml["seconds"], 3) if ok else None
    return out


def oracle_sample(H, n, nnz, n_b, prec, target_s):
    """Time the FP64 CPU oracle (unfused Alg. 1) on one block of n_b vectors for a few
    degree steps; returns its algorithmic GB/s under the same byte model."""
    import oracle as O
    from topi import random_phase_block
    from paper_1803_02156_amd import traffic

    lib = O.load_library()
    X = random_phase_block(n, n_b, 4242)
    lo, hi = O.gershgorin_bounds(H)
    al, be = O.scale_factors(lo, hi)
    # calibrate: a degree-4 filter, then scale the degree to the time budget
    t0 = time.perf_counter()
    O.chebyshev_filter(H, al, be, np.ones(5), X, n_b)
    t4 = time.perf_counter() - t0
    per_step = max(t4 / 3.0, 1e-6)
    n_p = int(max(5, min(400, target_s / per_step)))
    gam = np.ones(n_p + 1)
    t0 = time.perf_counter()
    O.chebyshev_filter(H, al, be, gam, X, n_b)
    dt = time.perf_counter() - t0
    # bytes of the same filter under the FP64 model (the oracle computes in FP64)
    nbytes = traffic.filter_bytes(n, nnz, n_b, n_b, n_p, 0)
    return {
        "value": nbytes / dt / 1e9, "unit": "GB/s", "cores": int(lib.orc_num_threads()),
        "kind": "oracle",
        "sample": f"one block of n_b={n_b} vectors, filter degree {n_p} (of the {n_p} steps "
                  f"{n_p - 2} fused-step equivalents), same matrix, FP64, {dt:.1f} s",
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "layout is a design note, not a measured path", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1803_02156_amd as P
    from paper_1803_02156_amd import traffic
    from topi import random_phase_block, topi_csr

    if not torch.cuda.is_available():
        print("no ROCm GPU visible", file=sys.stderr)
        sys.exit(1)
    P.load()
    Nx, Ny, Nz = (int(v) for v in args.lattice.split("x"))
    n_s, n_b, n_p, prec = args.n_s, args.n_b, args.n_p, args.prec

    t0 = time.perf_counter()
    H = topi_csr(Nx, Ny, Nz, m=1.0, W=args.W, t=1.0, seed=1002)
    n, nnz = len(H[0]) - 1, len(H[1])
    from paper_1803_02156_amd.ordering import lattice_row_order
    order = lattice_row_order(Nx, Ny, Nz) if args.order == "lattice" else None
    M = P.chebfd_matrix_build(*H, C=32, sigma=256, prec=prec, order=order)
    lo, hi = P.chebfd_bounds(M)
    lam = 0.1  # search interval [-0.1, 0.1] in H's units (the filter's cost does not depend on it)
    al, be, gam = P.chebfd_coefficients(lo, hi, -lam, lam, n_p)
    X0 = random_phase_block(n, n_s, 44)
    x0 = torch.empty((n_s, n), dtype=torch.complex128, device="cuda")
    x0.copy_(torch.from_numpy(np.ascontiguousarray(X0.T)))
    del X0
    xb0 = P.chebfd_pack(M, x0.T, n_b)
    del x0
    xy = torch.empty_like(xb0)
    work = P.FilterWork(M, n_b, n_p, n_s, moments=True)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    print(f"# setup {setup_s:.1f} s: n={n} nnz={nnz} bounds=[{lo:.4f},{hi:.4f}]", file=sys.stderr, flush=True)

    stream = torch.cuda.current_stream()

    def step():
        xy.copy_(xb0)   # fresh start block each step (the filter overwrites X by Y)
        P.chebfd_filter(M, al, be, gam, n_s, n_b, xy, work=work)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # timed region: K steps (restore the start block -- 2 n n_s elements copied, under
    # 0.1% of a step -- then the full filter); events on the stream the kernels run on
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    filt_ms = ev0.elapsed_time(ev1) / args.steps

    fbytes = traffic.filter_bytes(n, nnz, n_s, n_b, n_p, prec)
    gbs = fbytes / (filt_ms * 1e-3) / 1e9
    gflops = traffic.filter_flops(n, n_s, n_p, nnz / n) / (filt_ms * 1e-3) / 1e9
    # the fused step also timed alone: op_launches back-to-back launches on three blocks
    # of the start block (no partials of a previous launch to reduce), events on the stream
    xv = xy.view(n_s // n_b, n, n_b)
    opw = P.device_buffer(P.chebfd_filter_query(M, n_b))
    opb = opw.numel()
    P.chebfd_op(M, al, be, gam[3], n_b, xv[0], xv[1], xv[2], opw, opb)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.op_launches):
        P.chebfd_op(M, al, be, gam[3], n_b, xv[0], xv[1], xv[2], opw, opb)
    e1.record(stream)
    torch.cuda.synchronize()
    op_alone_s = e0.elapsed_time(e1) * 1e-3 / args.op_launches
    # the kernel's average launch over the timed region: every launch of a filter is
    # this kernel (n_p - 2 fused steps and the two start launches of each block)
    avg_launch_s = filt_ms * 1e-3 / ((n_s // n_b) * n_p)
    r, w = traffic.step_bytes(n, nnz, n_b, prec)
    achieved = (r + w) / avg_launch_s / 1e9
    kind = P.chebfd_step_kernel(M, n_b)
    hbm = counter_traffic(kind, prec, n_b, args.lattice, args.order)
    del opw
    # the orthogonalisation's Gram product Y^H Y over the whole search block (FP64 MFMA)
    P.chebfd_gram(xy.view(n_s // n_b, n, n_b), xy.view(n_s // n_b, n, n_b))
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(5):
        P.chebfd_gram(xy.view(n_s // n_b, n, n_b), xy.view(n_s // n_b, n, n_b))
    e1.record(stream)
    torch.cuda.synchronize()
    gram_ms = e0.elapsed_time(e1) / 5
    gram_tflops = 8.0 * n * n_s * n_s / (gram_ms * 1e-3) / 1e12

    # attainable HBM bandwidth: copy probe over 2 x 2 GiB (the STREAM analogue of Table 2)
    cnt = 1 << 28
    pa = torch.empty(cnt, dtype=torch.float64, device="cuda")
    pb = torch.ones(cnt, dtype=torch.float64, device="cuda")
    P.chebfd_probe_stream(0, pa, pb)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(10):
        P.chebfd_probe_stream(0, pa, pb)
    e1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 10 * 2 * 8 * cnt / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del pa, pb

    mixed = None
    if prec == 0 and not args.no_mixed_filter:
        mixed = mixed_filter_leg(P, H, order, args.lattice, args.order, n_s, n_b, n_p, args.steps)
        print(f"# mixed filter: {mixed['value']:.0f} GB/s, {mixed['avg_launch_us']:.1f} us per step",
              file=sys.stderr, flush=True)

    solve = None
    if not args.no_solve:
        del xy, xb0, work
        torch.cuda.empty_cache()
        solve = time_to_converged(P, H, Nx, Ny, Nz, args.W, n_s, n_b, n_p, args.solve_count, order,
                                  args.solve_prec)

    cpu = None
    if args.cpu_baseline_seconds > 0:
        try:
            cpu = oracle_sample(H, n, nnz, n_b, prec, args.cpu_baseline_seconds)
        except Exception as e:  # report, never hide the GPU result
            cpu = {"value": None, "unit": "GB/s", "cores": None, "kind": "oracle", "sample": f"failed: {e}"}

    out = {
        "metric": METRIC,
        "value": round(gbs, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(filt_ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128" if prec == 0 else "c64",
        "data": "synthetic",
        "config": {
            "workload": f"Topi-{Nx}-{Ny}-{Nz} (n={n}, nnz={nnz}, W={args.W}), "
                        f"{'FP64' if prec == 0 else 'mixed c64'} full filter, n_s={n_s}, n_b={n_b}, "
                        f"n_p={n_p}, SELL-32-256, {args.order} row order",
            "n": n, "n_s": n_s, "n_b": n_b, "n_p": n_p, "prec": "fp64" if prec == 0 else "mixed",
            "row_order": args.order,
        },
        "pct_of_hbm_peak": round(100.0 * gbs / HBM_PEAK_GBS, 2),
        "gflops": round(gflops, 1),
        "copy_probe_gbs": round(copy_gbs, 1),
        "pct_of_copy_probe": round(100.0 * gbs / copy_gbs, 2),
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": hbm,
            "kernel": f"{STEP_KERNELS[kind][0]}_kernel<{'double' if prec == 0 else 'float'},{n_b},kModeStep>",
            "bytes_per_launch": r + w, "avg_launch_us": round(avg_launch_s * 1e6, 3),
            "fused_step_alone_us": round(op_alone_s * 1e6, 3),
            "kernel_source_sha256_16": kernel_source_hash(kind),
        },
        "gram": {"kernel": "gram_kernel (FP64 MFMA 16x16x4)", "shape": f"{n} x {n_s} x {n_s} complex",
                 "ms": round(gram_ms, 3), "tflops": round(gram_tflops, 2),
                 "frac_of_fp64_mfma_peak": round(gram_tflops / 78.6, 4)},
        "filter_mixed": mixed,
        "time_to_converged": solve,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
