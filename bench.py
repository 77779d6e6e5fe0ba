#!/usr/bin/env python3
"""Benchmark of the ChebFD polynomial filter on one MI355X.

Headline workload: the Topi-256-256-128 lattice Hamiltonian (n = 33554432,
13 non-zeros per row, m = 1, disorder W = 1, complex double, SELL-32-256,
lattice row order), the largest configuration one GPU holds.  One step = the
filter polynomial of degree n_p = 100 applied to one block of n_b = 32 search
vectors (Alg. 1: two start launches and n_p - 2 fused chebfd_op steps, with
the dot products and the filtered-block update), from a fresh random-phase
start block.  The n_s = 256 search space is 8 such blocks, which are
independent (Alg. 2).  Inputs are synthetic and resident in HBM before the
timed region.

Prints one JSON line: `value` = the paper's minimum-traffic bytes of the
filter (Sect. 3.4, Eq. 2) per second; the roofline of the fused step kernel
(its average launch over the timed region, HIP events on the launch stream);
the unfused filter on the same block (SpMMV, dot and axpby as separate calls,
the GHOST-nofuse comparison of Sect. 3.2); the same filter with c64 block
vectors; the FP64 MFMA Gram product Y^H Y of a 256-vector search space; the
time to converged Ritz pairs on the 64x64x32 lattice in FP64 and mixed
precision with the heuristic's (n_p, n_s) and in mixed precision with the
learned (n_p, n_s); and the FP64 CPU oracle timed on bounded samples on the
host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E, published
FP64_MFMA_PEAK_TFLOPS = 78.6
METRIC = "Cheb filter HBM GB/s (% of peak); time to converged pairs, plain vs mixed"


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--lattice", type=str, default="256x256x128")
    ap.add_argument("--W", type=float, default=1.0)
    ap.add_argument("--n_b", type=int, default=32)
    ap.add_argument("--n_p", type=int, default=100)
    ap.add_argument("--prec", type=int, default=0, help="0 = FP64, 1 = mixed (c64 storage)")
    ap.add_argument("--order", choices=("lattice", "natural"), default="lattice",
                    help="row order at ingest: lattice boxes/pencils (one box per XCD) or the natural order")
    ap.add_argument("--op-launches", type=int, default=20, help="launches of the fused step timed alone")
    ap.add_argument("--no-unfused", action="store_true", help="skip the unfused filter leg")
    ap.add_argument("--mixed-n_b", type=int, default=32, help="block width of the c64 filter leg (0 skips it)")
    ap.add_argument("--gram-n_s", type=int, default=256, help="search-space size of the Gram leg (0 skips it)")
    ap.add_argument("--solve-lattice", type=str, default="64x64x32",
                    help="lattice of the time-to-converged leg ('' skips it)")
    ap.add_argument("--solve-W", type=float, default=1.0)
    ap.add_argument("--solve-count", type=float, default=100.0,
                    help="eigenvalue count the symmetric search interval is sized for")
    ap.add_argument("--solve-n_b", type=int, default=32)
    ap.add_argument("--solve-runs", type=str, default="fp64_heuristic,mixed_heuristic,mixed_learned,mixed_heuristic_tsqr",
                    help="comma-separated subset of the time-to-converged runs")
    ap.add_argument("--solve-n_s", type=int, default=0,
                    help="subspace size of every time-to-converged run (0: from the heuristic / the network)")
    ap.add_argument("--beyond-hbm-lattice", type=str, default="128x128x64",
                    help="lattice of the host-resident search-space leg ('' skips it)")
    ap.add_argument("--cpu-baseline-seconds", type=float, default=15.0,
                    help="target CPU time of each oracle sample (0 disables)")
    return ap.parse_args()


def log(msg):
    print(f"# {msg}", file=sys.stderr, flush=True)


# fused-step kernels (chebfd_step_kernel kinds): short name, source file
STEP_KERNELS = {0: ("cheb_lds", "filter_lds.hip"), 1: ("cheb_row", "filter_rows.hip"),
                2: ("cheb_multirow", "filter.hip"), 3: ("cheb_win", "filter_win.hip")}


def kernel_source_hash(kind: int) -> str:
    """Hash of the step kernel's source and the headers it includes."""
    h = hashlib.sha256()
    for name in (STEP_KERNELS[kind][1], "step_io.h", "kernels.h"):
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


class BlockFilter:
    """One n_b-vector block of the lattice matrix M: a device start block, a work
    block and timed filter applications (restore the start block, then filter)."""

    def __init__(self, P, M, n_b, n_p, lam=0.1, seed=44):
        import torch
        self.P, self.M, self.n_b, self.n_p = P, M, n_b, n_p
        lo, hi = P.chebfd_bounds(M)
        self.bounds = (lo, hi)
        # search interval [-lam, lam] in H's units (the filter's cost does not depend on it)
        self.al, self.be, self.gam = P.chebfd_coefficients(lo, hi, -lam, lam, n_p)
        self.x0 = P.chebfd_random_phase(M, n_b, n_b, seed)
        self.xy = torch.empty_like(self.x0)
        self.work = P.FilterWork(M, n_b, n_p, n_b, moments=True)
        self.stream = torch.cuda.current_stream()

    def run(self, steps, unfused=False):
        """Time `steps` steps; returns (ms per step, ms of the filter calls alone per step)."""
        import torch
        P = self.P
        fn = P.chebfd_filter_unfused if unfused else P.chebfd_filter
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(self.stream)
        for k in range(steps):
            self.xy.copy_(self.x0)   # fresh start block (the filter overwrites X by Y)
            ev[k][0].record(self.stream)
            fn(self.M, self.al, self.be, self.gam, self.n_b, self.n_b, self.xy, work=self.work)
            ev[k][1].record(self.stream)
        e1.record(self.stream)
        torch.cuda.synchronize()
        total = e0.elapsed_time(e1) / steps
        filt = sum(a.elapsed_time(b) for a, b in ev) / steps
        return total, filt

    def op_alone(self, launches):
        """Average duration of `launches` back-to-back chebfd_op launches (the Step kernel)."""
        import torch
        P = self.P
        opw = P.device_buffer(P.chebfd_filter_query(self.M, self.n_b))
        u, w, y = self.work.u, self.work.w, self.xy.view(self.M.n, self.n_b)
        P.chebfd_op(self.M, self.al, self.be, self.gam[3], self.n_b, u, w, y, opw, opw.numel())
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(self.stream)
        for _ in range(launches):
            P.chebfd_op(self.M, self.al, self.be, self.gam[3], self.n_b, u, w, y, opw, opw.numel())
        e1.record(self.stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e-3 / launches


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


def time_to_converged(P, lattice, W, n_b, target, n_s_fixed=0,
                      which=("fp64_heuristic", "mixed_heuristic", "mixed_learned", "mixed_heuristic_tsqr")):
    """Full ChebFD runs (filter, SVQB, Rayleigh-Ritz, residuals, restarts) on one
    matrix and interval: FP64 and mixed precision with the heuristic's (n_p, n_s)
    (the fallback rule), mixed precision with the learned (n_p, n_s), and mixed
    precision with the heuristic's choice and TSQR in place of SVQB.  Wall time
    from the first launch to the synchronised end; matrix build excluded."""
    import torch
    from paper_1803_02156_amd import predictor as PR
    from paper_1803_02156_amd.ordering import lattice_row_order
    from topi import topi_csr
    Nx, Ny, Nz = (int(v) for v in lattice.split("x"))
    H = topi_csr(Nx, Ny, Nz, m=1.0, W=W, t=1.0, seed=1002)
    order = lattice_row_order(Nx, Ny, Nz)
    M64 = P.chebfd_matrix_build(*H, prec=0, order=order)
    M32 = P.chebfd_matrix_build(*H, prec=1, order=order)
    delta, cnt = interval_for_count(P, M64, target)
    pred = PR.load(PR.DEFAULT_WEIGHTS)
    f, cnt_f, _, _ = P.chebfd_features(M64, -delta, delta, 7)
    hp, hs = PR.choose(None, f, cnt_f, pred["kappa"])
    lp, ls = PR.choose(pred, f, cnt_f, pred["kappa"])
    if n_s_fixed > 0:
        hs = ls = n_s_fixed
    out = {"workload": f"Topi-{Nx}-{Ny}-{Nz} (n={M64.n}, W={W}), interval [-{delta:.6g}, {delta:.6g}] "
                       f"(KPM count estimate {cnt:.1f}, 2048 moments), n_b={n_b}, max 12 iterations",
           "interval": [-delta, delta], "count_est_kpm": cnt, "count_est_features": cnt_f,
           "heuristic": {"n_p": hp, "n_s": hs, "kappa": pred["kappa"]}, "learned": {"n_p": lp, "n_s": ls}}
    runs = {}
    for name, M, n_p, n_s, orth in (("fp64_heuristic", M64, hp, hs, "svqb"), ("mixed_heuristic", M32, hp, hs, "svqb"),
                                    ("mixed_learned", M32, lp, ls, "svqb"),
                                    ("mixed_heuristic_tsqr", M32, hp, hs, "tsqr")):
        if name not in which:
            continue
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = P.chebfd_solve(M, M64, -delta, delta, n_s, n_p, n_b, seed=43, max_iter=12, want_vectors=False,
                           orth=orth)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        nf, st = r.n_found, r.stats
        runs[name] = r
        out[name] = {
            "seconds": round(dt, 3), "status": r.status, "iterations": st.iterations, "n_found": nf,
            "n_p": n_p, "n_s": n_s, "orth": orth, "max_resid": float(np.max(r.resid[:nf])) if nf else None,
            "tol": 1e-9 if M is M64 else 1e-7,
            "t_filter": round(st.t_filter, 3), "t_orth": round(st.t_orth, 3), "t_rr": round(st.t_rr, 3),
            "t_resid": round(st.t_resid, 3),
            "filter_gbs": round(st.filter_bytes / st.t_filter / 1e9, 1) if st.t_filter > 0 else None,
        }
        log(f"solve {name} (n_p {n_p}, n_s {n_s}): {dt:.2f} s, status {r.status}, {st.iterations} iterations, "
            f"{nf} pairs")
    ref = runs.get("fp64_heuristic")
    for name in ("mixed_heuristic", "mixed_learned", "mixed_heuristic_tsqr"):
        if name not in runs or ref is None:
            continue
        r = runs[name]
        o = out[name]
        o["all_pairs_of_fp64_run"] = bool(r.status == 0 and ref.status == 0 and r.n_found >= ref.n_found > 0)
        if r.n_found == ref.n_found and r.n_found > 0:
            o["max_abs_dtheta_vs_fp64"] = float(np.max(np.abs(np.sort(r.theta[:r.n_found]) -
                                                             np.sort(ref.theta[:ref.n_found]))))
        o["speedup_vs_fp64_heuristic"] = round(out["fp64_heuristic"]["seconds"] / o["seconds"], 3)
    del M64, M32
    return out, H


def beyond_hbm(P, lattice, n_b=32, n_s=128, degrees=(10, 30, 100)):
    """The filter on a search space held in pinned host memory (blocks streamed
    through two device staging blocks, Sect. 3.5 / Fig. 6) against the same
    filter on a device-resident search space, for several filter degrees."""
    import torch
    from paper_1803_02156_amd.ordering import lattice_row_order
    from topi import topi_csr
    Nx, Ny, Nz = (int(v) for v in lattice.split("x"))
    H = topi_csr(Nx, Ny, Nz, m=1.0, W=1.0, t=1.0, seed=1002)
    M = P.chebfd_matrix_build(*H, prec=0, order=lattice_row_order(Nx, Ny, Nz))
    del H
    lo, hi = P.chebfd_bounds(M)
    xd = P.chebfd_random_phase(M, n_s, n_b, 45)
    xh = torch.empty(xd.shape, dtype=xd.dtype, pin_memory=True)
    xh.copy_(xd)
    x0 = xd.clone()
    out = {"workload": f"Topi-{Nx}-{Ny}-{Nz} (n={M.n}), FP64, n_s={n_s} ({n_s // n_b} blocks of n_b={n_b}, "
                       f"{xh.numel() * 16 / 2**30:.1f} GiB in pinned host memory)", "runs": []}
    for n_p in degrees:
        al, be, gam = P.chebfd_coefficients(lo, hi, -0.1, 0.1, n_p)
        work = P.FilterWork(M, n_b, n_p, n_s, moments=True)
        P.chebfd_filter(M, al, be, gam, n_s, n_b, xd, work=work)     # warm-up
        xd.copy_(x0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P.chebfd_filter(M, al, be, gam, n_s, n_b, xd, work=work)
        torch.cuda.synchronize()
        t_dev = time.perf_counter() - t0
        t0 = time.perf_counter()
        P.chebfd_filter_streamed(M, al, be, gam, n_s, n_b, xh)
        torch.cuda.synchronize()
        t_host = time.perf_counter() - t0
        same = bool(torch.equal(xh, xd.cpu()))
        xh.copy_(x0)
        xd.copy_(x0)
        out["runs"].append({"n_p": n_p, "device_s": round(t_dev, 4), "host_resident_s": round(t_host, 4),
                            "slowdown": round(t_host / t_dev, 3), "equal_results": same})
        log(f"beyond HBM n_p={n_p}: device {t_dev:.3f} s, host-resident {t_host:.3f} s")
        del work
    del xd, xh, x0, M
    torch.cuda.empty_cache()
    return out


def cpu_info():
    model = platform.processor() or None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable,
            "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS")}


def oracle_filter_rate(H, n_b, target_s, threads=None):
    """The FP64 CPU oracle (unfused Alg. 1) on one block of n_b vectors for a few
    degree steps of the given matrix; its rate under the same byte model."""
    import oracle as O
    from topi import random_phase_block
    from paper_1803_02156_amd import traffic

    lib = O.load_library()
    nthreads0 = lib.orc_num_threads()
    if threads:
        lib.orc_set_num_threads(threads)
    try:
        n, nnz = len(H[0]) - 1, len(H[1])
        X = random_phase_block(n, n_b, 4242)
        lo, hi = O.gershgorin_bounds(H)
        al, be = O.scale_factors(lo, hi)
        # calibrate with a degree-3 filter, then scale the degree to the time budget
        t0 = time.perf_counter()
        O.chebyshev_filter(H, al, be, np.ones(4), X, n_b)
        per_step = max((time.perf_counter() - t0) / 3.0, 1e-6)
        n_p = int(max(3, min(400, target_s / per_step)))
        t0 = time.perf_counter()
        O.chebyshev_filter(H, al, be, np.ones(n_p + 1), X, n_b)
        dt = time.perf_counter() - t0
        nbytes = traffic.filter_bytes(n, nnz, n_b, n_b, n_p, 0)
        used = lib.orc_num_threads()
    finally:
        lib.orc_set_num_threads(nthreads0)
    return {"value": nbytes / dt / 1e9, "unit": "GB/s", "cores": int(used), "seconds": round(dt, 2),
            "n_p": n_p, "gflops": traffic.filter_flops(n, n_b, n_p, nnz / n) / dt / 1e9}


def oracle_small_solve():
    """Time to converged pairs of the oracle's full FP64 solve on the 16x16x8
    configuration (interval [-0.05, 0.05], n_s = n_b = 32, n_p = 200)."""
    import oracle as O
    from topi import random_phase_block, topi_csr
    H = topi_csr(16, 16, 8, m=1.0, W=1.0, seed=1001)
    X0 = random_phase_block(8192, 32, 43)
    t0 = time.perf_counter()
    r = O.chebfd_solve(H, -0.05, 0.05, 32, 200, 32, X0, refill_seed=44)
    dt = time.perf_counter() - t0
    return {"seconds": round(dt, 3), "status": r.status, "iterations": r.iterations, "n_found": r.n_found,
            "cores": int(O.load_library().orc_num_threads())}, H


def gpu_small_solve(P, H):
    import torch
    M = P.chebfd_matrix_build(*H, prec=0)
    P.chebfd_solve(M, M, -0.05, 0.05, 32, 200, 32, seed=43, want_vectors=False)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = P.chebfd_solve(M, M, -0.05, 0.05, 32, 200, 32, seed=43, want_vectors=False)
    torch.cuda.synchronize()
    return {"seconds": round(time.perf_counter() - t0, 3), "status": r.status, "iterations": r.stats.iterations,
            "n_found": r.n_found}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "layout is a design note, not a measured path", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1803_02156_amd as P
    from paper_1803_02156_amd import traffic
    from paper_1803_02156_amd.ordering import lattice_row_order
    from topi import topi_csr

    if not torch.cuda.is_available():
        print("no ROCm GPU visible", file=sys.stderr)
        sys.exit(1)
    P.load()
    Nx, Ny, Nz = (int(v) for v in args.lattice.split("x"))
    n_b, n_p, prec = args.n_b, args.n_p, args.prec

    t0 = time.perf_counter()
    H = topi_csr(Nx, Ny, Nz, m=1.0, W=args.W, t=1.0, seed=1002)
    n, nnz = len(H[0]) - 1, len(H[1])
    order = lattice_row_order(Nx, Ny, Nz) if args.order == "lattice" else None
    log(f"matrix generated: n={n} nnz={nnz} ({time.perf_counter() - t0:.1f} s)")
    M = P.chebfd_matrix_build(*H, C=32, sigma=256, prec=prec, order=order)
    bf = BlockFilter(P, M, n_b, n_p)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    log(f"setup {setup_s:.1f} s, bounds [{bf.bounds[0]:.4f}, {bf.bounds[1]:.4f}]")

    if args.warmup:
        bf.run(args.warmup)
    # timed region: K steps, each = restore the start block (2 n n_b elements, ~0.4% of a
    # step, not counted as algorithmic bytes) + the degree-n_p filter on the block
    step_ms, filt_ms = bf.run(args.steps)
    log(f"filter: {step_ms:.2f} ms per step ({filt_ms:.2f} ms in the filter calls)")
    fbytes = traffic.filter_bytes(n, nnz, n_b, n_b, n_p, prec)
    gbs = fbytes / (step_ms * 1e-3) / 1e9
    gflops = traffic.filter_flops(n, n_b, n_p, nnz / n) / (step_ms * 1e-3) / 1e9
    # the fused step kernel: every launch of a filter call is that kernel (n_p - 2
    # recurrence steps and the two start launches), timed by the per-step events
    avg_launch_s = filt_ms * 1e-3 / n_p
    r, w = traffic.step_bytes(n, nnz, n_b, prec)
    achieved = (r + w) / avg_launch_s / 1e9
    kind = P.chebfd_step_kernel(M, n_b)
    op_alone_s = bf.op_alone(args.op_launches)

    unfused = None
    if not args.no_unfused:
        k = max(1, min(args.steps, 5))
        bf.run(1, unfused=True)
        u_step, u_filt = bf.run(k, unfused=True)
        ur, uw = traffic.unfused_step_bytes(n, nnz, n_b, prec)
        ubytes = traffic.unfused_filter_bytes(n, nnz, n_b, n_b, n_p, prec)
        unfused = {"ms_per_step": round(u_step, 3), "steps": k,
                   "value": round(fbytes / (u_step * 1e-3) / 1e9, 2), "unit": "GB/s",
                   "note": "value: the fused filter's algorithmic bytes per second of the unfused run",
                   "gflops": round(traffic.filter_flops(n, n_b, n_p, nnz / n) / (u_step * 1e-3) / 1e9, 1),
                   "own_bytes_per_step": ubytes, "own_gbs": round(ubytes / (u_step * 1e-3) / 1e9, 2),
                   "own_bytes_per_recurrence_step": ur + uw,
                   "fused_speedup": round(u_step / step_ms, 3)}
        log(f"unfused filter: {u_step:.2f} ms per step (fused {step_ms:.2f} ms: x{u_step / step_ms:.2f})")

    # attainable HBM bandwidth (the STREAM analogue of Table 2) over arrays of 4 GiB: the
    # plain copy, the non-temporal copy (four 16-byte elements per thread), a read-only
    # pass and the triad a = b + s c (two reads per write, about the step's own mix)
    cnt = 1 << 29
    pa = torch.empty(cnt, dtype=torch.float64, device="cuda")
    pb = torch.ones(cnt, dtype=torch.float64, device="cuda")
    pc = torch.ones(cnt, dtype=torch.float64, device="cuda")
    probes = {}
    for pkind, name, nbytes in ((0, "copy", 16 * cnt), (2, "copy_nt", 16 * cnt), (3, "read", 8 * cnt),
                                (1, "triad", 24 * cnt)):
        P.chebfd_probe_stream(pkind, pa, pb, pc)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(bf.stream)
        for _ in range(10):
            P.chebfd_probe_stream(pkind, pa, pb, pc)
        e1.record(bf.stream)
        torch.cuda.synchronize()
        probes[name] = round(10 * nbytes / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
    copy_gbs = max(probes["copy"], probes["copy_nt"])
    log(f"probes: {probes}")
    del pa, pb, pc
    del bf, M
    torch.cuda.empty_cache()

    mixed = None
    if prec == 0 and args.mixed_n_b > 0:
        mb = args.mixed_n_b
        M32 = P.chebfd_matrix_build(*H, C=32, sigma=256, prec=1, order=order)
        bm = BlockFilter(P, M32, mb, n_p)
        bm.run(1)
        k = max(1, min(args.steps, 5))
        m_step, m_filt = bm.run(k)
        mbytes = traffic.filter_bytes(n, nnz, mb, mb, n_p, 1)
        m_avg = m_filt * 1e-3 / n_p
        rm, wm = traffic.step_bytes(n, nnz, mb, 1)
        mkind = P.chebfd_step_kernel(M32, mb)
        mixed = {"value": round(mbytes / (m_step * 1e-3) / 1e9, 2), "unit": "GB/s", "ms_per_step": round(m_step, 3),
                 "n_b": mb, "steps": k, "pct_of_hbm_peak": round(100.0 * mbytes / (m_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 2),
                 "gflops": round(traffic.filter_flops(n, mb, n_p, nnz / n) / (m_step * 1e-3) / 1e9, 1),
                 "kernel": f"{STEP_KERNELS[mkind][0]}_kernel<float,{mb},kModeStep>",
                 "avg_launch_us": round(m_avg * 1e6, 3), "bytes_per_launch": rm + wm,
                 "frac": round((rm + wm) / m_avg / 1e9 / HBM_PEAK_GBS, 4),
                 "traffic": counter_traffic(mkind, 1, mb, args.lattice, args.order),
                 "kernel_source_sha256_16": kernel_source_hash(mkind)}
        log(f"mixed filter n_b={mb}: {mixed['value']:.0f} GB/s, {mixed['avg_launch_us']:.1f} us per launch")
        del bm

        gram = None
        if args.gram_n_s > 0:
            # the orthogonalisation's Gram product Y^H Y of a c64 search space (cfg: c64
            # storage, FP64 products), FP64 MFMA; the Hermitian product forms its upper triangle
            ns = args.gram_n_s
            Y = P.chebfd_random_phase(M32, ns, mb, 99)
            P.chebfd_gram(Y, Y)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            stream = torch.cuda.current_stream()
            e0.record(stream)
            for _ in range(3):
                P.chebfd_gram(Y, Y)
            e1.record(stream)
            torch.cuda.synchronize()
            gram_ms = e0.elapsed_time(e1) / 3
            # flops of the Hermitian product's distinct entries (upper triangle and diagonal)
            useful = 8.0 * n * ns * (ns + 1) / 2
            gram = {"kernel": "gram_kernel (FP64 MFMA 16x16x4)", "shape": f"{n} x {ns} x {ns} complex (c64 in)",
                    "ms": round(gram_ms, 3), "tflops": round(useful / (gram_ms * 1e-3) / 1e12, 2),
                    "frac_of_fp64_mfma_peak": round(useful / (gram_ms * 1e-3) / 1e12 / FP64_MFMA_PEAK_TFLOPS, 4),
                    "flops_counted": "8 n n_s (n_s + 1) / 2: the distinct entries of the Hermitian S"}
            log(f"gram: {gram_ms:.1f} ms, {gram['tflops']} TFLOP/s")
            # TSQR of the same search space (the alternative orthogonalisation): panels of
            # min(n_b, 32) columns, block Gram-Schmidt twice + a Householder tree per panel
            P.chebfd_tsqr(Y)
            torch.cuda.synchronize()
            e0.record(stream)
            P.chebfd_tsqr(Y)
            e1.record(stream)
            torch.cuda.synchronize()
            tsqr_ms = e0.elapsed_time(e1)
            gram["tsqr_ms"] = round(tsqr_ms, 3)
            gram["tsqr_note"] = ("chebfd_tsqr of the same c64 block (Q c64, R FP64); one TSQR replaces "
                                 "the two SVQB steps of an iteration (each a Gram, a small eigensolve, an update)")
            log(f"tsqr: {tsqr_ms:.1f} ms")
            del Y
        del M32
        torch.cuda.empty_cache()
    else:
        gram = None

    solve = None
    if args.solve_lattice:
        solve, H_small = time_to_converged(P, args.solve_lattice, args.solve_W, args.solve_n_b, args.solve_count,
                                           args.solve_n_s, tuple(args.solve_runs.split(",")))
        torch.cuda.empty_cache()

    hostres = None
    if args.beyond_hbm_lattice:
        hostres = beyond_hbm(P, args.beyond_hbm_lattice)

    cpu = None
    if args.cpu_baseline_seconds > 0:
        try:
            s1 = oracle_filter_rate(H, n_b, args.cpu_baseline_seconds)
            log(f"oracle: {s1['value']:.1f} GB/s on {s1['cores']} threads")
            cpu = {"value": round(s1["value"], 3), "unit": "GB/s", "cores": s1["cores"], "kind": "oracle",
                   "sample": f"one block of n_b={n_b} vectors of the same matrix, filter degree {s1['n_p']} "
                             f"({s1['seconds']} s), FP64, unfused Alg. 1 in C with OpenMP",
                   "gflops": round(s1["gflops"], 2), **cpu_info()}
            del H
            if solve is not None:
                s2 = oracle_filter_rate(H_small, n_b, min(10.0, args.cpu_baseline_seconds), threads=1)
                cpu["one_thread"] = {"value": round(s2["value"], 3), "unit": "GB/s",
                                     "sample": f"Topi-{args.solve_lattice}, one block of n_b={n_b}, "
                                               f"degree {s2['n_p']} ({s2['seconds']} s)"}
            o, Hs = oracle_small_solve()
            g = gpu_small_solve(P, Hs)
            cpu["time_to_converged_small"] = {
                "workload": "Topi-16-16-8 (n=8192, W=1), [-0.05, 0.05], n_s=n_b=32, n_p=200, FP64",
                "oracle": o, "gpu": g}
        except Exception as e:  # report, never hide the GPU result
            cpu = {"value": None, "unit": "GB/s", "cores": None, "kind": "oracle", "sample": f"failed: {e}"}

    out = {
        "metric": METRIC,
        "value": round(gbs, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(step_ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128" if prec == 0 else "c64",
        "data": "synthetic",
        "config": {
            "workload": f"Topi-{Nx}-{Ny}-{Nz} (n={n}, nnz={nnz}, W={args.W}), "
                        f"{'FP64' if prec == 0 else 'mixed c64'}; one step = the degree-{n_p} filter on one "
                        f"block of n_b={n_b} vectors (Alg. 1; one of the n_s/n_b independent blocks of Alg. 2), "
                        f"SELL-32-256, {args.order} row order",
            "n": n, "nnz": nnz, "n_b": n_b, "n_p": n_p, "prec": "fp64" if prec == 0 else "mixed",
            "row_order": args.order, "setup_s": round(setup_s, 1),
        },
        "pct_of_hbm_peak": round(100.0 * gbs / HBM_PEAK_GBS, 2),
        "gflops": round(gflops, 1),
        "copy_probe_gbs": round(copy_gbs, 1),
        "stream_probes_gbs": probes,
        "pct_of_copy_probe": round(100.0 * gbs / copy_gbs, 2),
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": counter_traffic(kind, prec, n_b, args.lattice,
                                                                                  args.order),
            "kernel": f"{STEP_KERNELS[kind][0]}_kernel<{'double' if prec == 0 else 'float'},{n_b},kModeStep>",
            "bytes_per_launch": r + w, "avg_launch_us": round(avg_launch_s * 1e6, 3),
            "fused_step_alone_us": round(op_alone_s * 1e6, 3),
            "kernel_source_sha256_16": kernel_source_hash(kind),
        },
        "unfused": unfused,
        "filter_mixed": mixed,
        "gram": gram,
        "time_to_converged": solve,
        "beyond_hbm": hostres,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
