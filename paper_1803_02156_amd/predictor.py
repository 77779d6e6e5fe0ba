"""Learned choice of the filter degree n_p and the subspace size n_s.

The paper sets n_p and n_s by hand (Sect. 2: n_s somewhat above the number of
wanted eigenpairs; Sect. 2.1: n_p around 10^3 for its matrices) and notes that
the filter's dot products are KPM moments, i.e. a cheap picture of the
spectrum (Sect. 2).  This module turns that picture into the two parameters:

* features: ``chebfd_features`` (256 normalised moments from 16 random-phase
  vectors plus the scaled interval [a~, b~]);
* the fallback heuristic of ``chebfd_choose_params`` (n_p = kappa / delta,
  n_s = 2 n_hat);
* a 258-128-128-2 network trained with the library's own device kernels
  (``chebfd_mlp_grad`` / ``chebfd_mlp_adam``) on runs of the method itself.

Labels: for each instance a small grid of (n_p, n_s) around the heuristic is
solved (or, adaptively, n_p is doubled from the heuristic's until the solver
finds pairs, then one more doubling and one wider subspace are tried), and the
label is the run with the least deterministic work
``iters (n_p n_s nnz + c_orth n n_s^2)`` among the runs that converged with the
full eigenvalue count; the network regresses the standardised logs of two
scale-free ratios of that point, n_p delta~ (delta~ the half width of the
scaled interval) and n_s / max(2 n_hat, n_b) (n_hat the count estimate; the
heuristic's own n_s before rounding): the interval and the count estimate
already carry the matrix size, so the ratios learnt on small lattices transfer
to large ones.  The heuristic's kappa is the
median n_p delta~ of the training labels.

Every computation runs in libchebfd; this file only orchestrates runs and
stores their results (numpy on the host).
"""
from __future__ import annotations

import json
import math
import os
import time
from dataclasses import dataclass

import numpy as np
import torch

from . import _abi
from . import chebfd as P

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "data", "predictor.npz")

C_ORTH = 8.0          # relative weight of the dense O(n n_s^2) work per iteration
N_B = 32


@dataclass
class Instance:
    dims: tuple
    m: float
    W: float
    half_width: float      # search interval [-hw, hw] in H's units
    seed: int
    target: float = 0.0    # eigenvalue count the interval was sized for (0: half_width drawn directly)


def sample_instance(rng: np.random.Generator, ext_lo: int, ext_hi: int, seed: int,
                    count_range=None) -> Instance:
    """A Topi instance: extents in [ext_lo, ext_hi] with a random aspect ratio,
    m ~ U[0.5, 2.5], W ~ U[0, 3].  The interval half width is ~ U[0.01, 0.1], or,
    with count_range, sized later (``size_interval``) for a count ~ U[count_range]:
    on small lattices most fixed-width windows near 0 hold no eigenvalue at all."""
    dims = tuple(int(v) for v in rng.integers(ext_lo, ext_hi + 1, 3))
    m, W = float(rng.uniform(0.5, 2.5)), float(rng.uniform(0.0, 3.0))
    if count_range is None:
        return Instance(dims=dims, m=m, W=W, half_width=float(rng.uniform(0.01, 0.1)), seed=int(seed))
    return Instance(dims=dims, m=m, W=W, half_width=0.0, seed=int(seed),
                    target=float(rng.uniform(*count_range)))


def size_interval(M, target: float, seed: int, n_steps: int = 256, R: int = 16) -> float:
    """Half width of the symmetric interval whose KPM count estimate (2 n_steps
    moments, Jackson-damped window) is `target` (bisection on the host)."""
    lo, hi = P.chebfd_bounds(M)
    al, be, _ = P.chebfd_coefficients(lo, hi, -1e-3, 1e-3, 1)
    mu = P.chebfd_kpm_moments(M, al, be, n_steps, R, seed)
    half = max(abs(lo), abs(hi))
    a, b = 1e-4 * half, 0.9 * half
    for _ in range(50):
        mid = 0.5 * (a + b)
        _, _, gc = P.chebfd_coefficients(lo, hi, -mid, mid, 2 * n_steps - 1)
        if M.n * float(np.dot(gc, mu)) < target:
            a = mid
        else:
            b = mid
    return 0.5 * (a + b)


def build(inst: Instance, prec: int = _abi.PREC_FP64):
    from topi import topi_csr
    H = topi_csr(*inst.dims, m=inst.m, W=inst.W, seed=inst.seed)
    return H, P.chebfd_matrix_build(*H, prec=prec)


def work_units(n: int, nnz: int, n_p: int, n_s: int, iters: int) -> float:
    """Deterministic cost of a run: filter row-column products plus the dense part."""
    return float(iters) * (n_p * n_s * (nnz / n) * n + C_ORTH * n * n_s * n_s)


def run(M, inst: Instance, n_p: int, n_s: int, max_iter: int = 12):
    t0 = time.perf_counter()
    r = P.chebfd_solve(M, M, -inst.half_width, inst.half_width, n_s, n_p, N_B, seed=43 + inst.seed,
                       max_iter=max_iter, want_vectors=False)
    torch.cuda.synchronize()
    return r, time.perf_counter() - t0


NP_FACTORS = (0.5, 1.0, 2.0, 4.0)


def grid(heur_np: int, heur_ns: int, count_est: float = 0.0):
    """Label grid around the heuristic's (n_p, n_s): n_p times 0.5, 1, 2, 4 and n_s
    one block below (when that still holds 1.2 n_hat and one block), at and one
    block above the heuristic's, clamped to the parameter rule's ranges."""
    nps = sorted({int(min(_abi.NP_MAX, max(_abi.NP_MIN, round(heur_np * f)))) for f in NP_FACTORS})
    nss = {heur_ns, min(512, heur_ns + N_B)}
    lower = heur_ns - N_B
    if lower >= max(N_B, math.ceil(1.2 * max(count_est, 0.0))):
        nss.add(lower)
    return [(a, b) for a in nps for b in sorted(nss)]


def next_adaptive_np(n_p: int, found: list, np_cap: int):
    """The next filter degree of the adaptive label search, or None to stop.

    The search doubles n_p while no run has converged with pairs; it stops at
    np_cap, and once a doubling found no more pairs than the run before it
    (that instance's window is not resolved by a higher degree within the
    iteration limit: its subspace or its interval is the problem)."""
    if 2 * n_p > np_cap:
        return None
    if len(found) >= 2 and found[-1] > 0 and found[-1] <= found[-2]:
        return None
    return 2 * n_p


def make_corpus(count: int, seed: int, ext_lo: int, ext_hi: int, kappa: float, count_range=None, log=print,
                adaptive: bool = False, start_np: int = 50, out: str | None = None):
    """Features, heuristic choice, grid runs and labels of `count` instances
    (written to `out` after every instance when given)."""
    rng = np.random.default_rng(seed)
    rows = []
    for k in range(count):
        inst = sample_instance(rng, ext_lo, ext_hi, seed * 100000 + k, count_range)
        H, M = build(inst)
        if inst.target > 0:
            inst.half_width = size_interval(M, inst.target, seed=1000 + k)
        n, nnz = M.n, len(H[1])
        f, cnt, al, be = P.chebfd_features(M, -inst.half_width, inst.half_width, seed=7 + k)
        a, b = f[256], f[257]
        hp, hs = P.chebfd_choose_params(float(a), float(b), cnt, N_B, kappa=kappa)
        results = []

        def solve(n_p, n_s):
            r, dt = run(M, inst, n_p, n_s)
            results.append(dict(n_p=n_p, n_s=n_s, status=r.status, iters=r.stats.iterations,
                                n_found=r.n_found, seconds=dt,
                                work=work_units(n, nnz, n_p, n_s, r.stats.iterations)))
            log(f"#   run n_p {n_p} n_s {n_s}: status {r.status}, {r.stats.iterations} it, "
                f"{r.n_found} pairs, {dt:.2f} s")
            return r.status == 0 and r.n_found > 0
        if adaptive:
            # double n_p from the heuristic's until a run converges with pairs (at
            # most 8 times the start, see next_adaptive_np), then one more
            # doubling and one wider subspace at that degree
            n_p = max(hp, start_np)
            np_cap = min(_abi.NP_MAX, 8 * n_p)
            found = []
            while n_p is not None:
                if solve(n_p, hs):
                    if 2 * n_p <= _abi.NP_MAX:
                        solve(2 * n_p, hs)
                    solve(n_p, min(512, hs + N_B))
                    break
                found.append(results[-1]["n_found"])
                n_p = next_adaptive_np(n_p, found, np_cap)
        else:
            for n_p, n_s in grid(hp, hs, cnt):
                solve(n_p, n_s)
        full = max(x["n_found"] for x in results)
        ok = [x for x in results if x["status"] == 0 and x["n_found"] == full]
        # no label where no run found a pair: the grid then says nothing about (n_p, n_s)
        best = min(ok, key=lambda x: x["work"]) if ok and full > 0 else None
        rows.append(dict(inst=inst.__dict__, n=n, nnz=nnz, features=f.tolist(), count_est=cnt,
                         heuristic=(hp, hs), runs=results, full_count=full,
                         label=None if best is None else (best["n_p"], best["n_s"])))
        log(f"# corpus {k + 1}/{count}: dims {inst.dims} n={n} count~{cnt:.1f} found {full} "
            f"heur ({hp},{hs}) label {rows[-1]['label']}")
        if out:
            with open(out + ".tmp", "w") as f:
                json.dump(rows, f)
            os.replace(out + ".tmp", out)
    return rows


def features_of(row: dict) -> np.ndarray:
    """The 258 network inputs of a corpus row.  Slot 0 holds log10(n) / 8, as
    chebfd_features writes it (the normalised moment mu~_0 it replaces is 1 by
    construction); rows stored before that convention get it from their n."""
    f = np.asarray(row["features"], dtype=np.float32).copy()
    f[0] = np.float32(np.log10(float(row["n"])) / 8.0)
    return f


def targets(rows: list) -> np.ndarray:
    """The regression targets of labelled corpus rows: (n_p delta~, n_s / max(2 n_hat, n_b))."""
    out = []
    for r in rows:
        a, b = float(r["features"][256]), float(r["features"][257])
        n_p, n_s = r["label"]
        out.append((n_p * (b - a) / 2.0, n_s / max(2.0 * float(r["count_est"]), float(N_B))))
    return np.array(out, dtype=np.float64)


def kappa_from_corpus(rows: list) -> float:
    """The heuristic's constant: the median n_p delta~ of the labels."""
    return float(np.median(targets(rows)[:, 0]))


def standardise(labels: np.ndarray):
    lg = np.log(labels.astype(np.float64))
    mean = lg.mean(axis=0)
    std = np.maximum(lg.std(axis=0), 1e-3)
    return (lg - mean) / std, mean, std


def init_params(seed: int) -> np.ndarray:
    """He-normal weights, zero biases, in the library's flat layout."""
    rng = np.random.default_rng(seed)
    shapes = [(_abi.MLP_HIDDEN, _abi.MLP_IN), (_abi.MLP_HIDDEN,), (_abi.MLP_HIDDEN, _abi.MLP_HIDDEN),
              (_abi.MLP_HIDDEN,), (_abi.MLP_OUT, _abi.MLP_HIDDEN), (_abi.MLP_OUT,)]
    parts = [rng.standard_normal(s).ravel() * math.sqrt(2.0 / s[1]) if len(s) == 2 else np.zeros(s)
             for s in shapes]
    return np.concatenate(parts).astype(np.float32)


def train(X: np.ndarray, T: np.ndarray, steps: int = 3000, lr: float = 1e-3, seed: int = 0, log=print):
    """Full-batch Adam on the device kernels; returns the flat parameters (numpy)."""
    p = torch.from_numpy(init_params(seed)).cuda()
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    x = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).cuda()
    t = torch.from_numpy(np.ascontiguousarray(T, dtype=np.float32)).cuda()
    for step in range(1, steps + 1):
        loss, g = P.chebfd_mlp_grad(p, x, t)
        P.chebfd_mlp_adam(p, g, m, v, step, lr=lr)
        if step % 500 == 0 or step == 1:
            log(f"# train step {step}: loss {loss.item():.4f}")
    return p.cpu().numpy()


def predict(params: np.ndarray, features: np.ndarray) -> np.ndarray:
    p = torch.from_numpy(np.ascontiguousarray(params, dtype=np.float32)).cuda()
    x = torch.from_numpy(np.ascontiguousarray(np.atleast_2d(features), dtype=np.float32)).cuda()
    return P.chebfd_mlp_forward(p, x).cpu().numpy()


def target_range(T: np.ndarray):
    """(t_lo, t_hi): the range of the log targets, to which the parameter rule
    holds the network's outputs (a network asked far outside it extrapolates)."""
    lg = np.log(T.astype(np.float64))
    return tuple(lg.min(axis=0)), tuple(lg.max(axis=0))


def save(path: str, params: np.ndarray, mean, std, kappa: float, meta: dict, t_lo=(0.0, 0.0),
         t_hi=(0.0, 0.0)):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.savez(path, params=params.astype(np.float32), t_mean=np.asarray(mean), t_std=np.asarray(std),
             kappa=np.asarray(kappa), meta=np.asarray(json.dumps(meta)), t_lo=np.asarray(t_lo),
             t_hi=np.asarray(t_hi))


def load(path: str = DEFAULT_WEIGHTS):
    z = np.load(path, allow_pickle=False)
    rng = (tuple(z["t_lo"]), tuple(z["t_hi"])) if "t_lo" in z.files else ((0.0, 0.0), (0.0, 0.0))
    return dict(params=z["params"], t_mean=tuple(z["t_mean"]), t_std=tuple(z["t_std"]),
                kappa=float(z["kappa"]), meta=json.loads(str(z["meta"])), t_lo=rng[0], t_hi=rng[1])


def choose(pred: dict | None, features: np.ndarray, count_est: float, kappa: float):
    """(n_p, n_s): the network's choice if `pred` is given, else the heuristic."""
    a, b = float(features[256]), float(features[257])
    if pred is None:
        return P.chebfd_choose_params(a, b, count_est, N_B, kappa=kappa)
    out = predict(pred["params"], features)[0]
    return P.chebfd_choose_params(a, b, count_est, N_B, out, kappa=kappa, t_mean=pred["t_mean"],
                                  t_std=pred["t_std"], t_lo=pred.get("t_lo", (0.0, 0.0)),
                                  t_hi=pred.get("t_hi", (0.0, 0.0)))


def evaluate(pred: dict, corpus: list, kappa: float, log=print):
    """Solve every instance with the heuristic's and with the network's (n_p, n_s);
    compare iterations, work, wall time and failures (a run that is not converged
    or finds fewer pairs than the instance's full count)."""
    out = []
    for k, row in enumerate(corpus):
        inst = Instance(**{**row["inst"], "dims": tuple(row["inst"]["dims"])})
        H, M = build(inst)
        f = features_of(row)
        res = {}
        for name, pr in (("heuristic", None), ("mlp", pred)):
            n_p, n_s = choose(pr, f, row["count_est"], kappa)
            r, dt = run(M, inst, n_p, n_s)
            res[name] = dict(n_p=n_p, n_s=n_s, status=r.status, iters=r.stats.iterations, n_found=r.n_found,
                             seconds=dt, work=work_units(M.n, len(H[1]), n_p, n_s, r.stats.iterations),
                             full_count_found=bool(r.n_found >= row["full_count"]),
                             failed=bool(r.status != 0 or r.n_found < row["full_count"]))
        out.append(dict(inst=row["inst"], full_count=row["full_count"], **res))
        log(f"# eval {k + 1}/{len(corpus)}: heur {res['heuristic']['n_p']},{res['heuristic']['n_s']} "
            f"it {res['heuristic']['iters']} {res['heuristic']['seconds']:.3f}s | mlp {res['mlp']['n_p']},"
            f"{res['mlp']['n_s']} it {res['mlp']['iters']} {res['mlp']['seconds']:.3f}s")
    return out


def summarise(ev: list) -> dict:
    def col(name, key):
        return np.array([e[name][key] for e in ev], dtype=np.float64)
    s = {"instances": len(ev)}
    for name in ("heuristic", "mlp"):
        s[name] = {"failures": int(sum(e[name]["failed"] for e in ev)),
                   "full_count_found": int(sum(e[name].get("full_count_found", not e[name]["failed"]) for e in ev)),
                   "not_converged": int(sum(e[name]["status"] != 0 for e in ev)) if all("status" in e[name] for e in ev)
                   else None,
                   "mean_iters": float(col(name, "iters").mean()),
                   "total_seconds": float(col(name, "seconds").sum()),
                   "total_work": float(col(name, "work").sum())}
    ok = [e for e in ev if not e["heuristic"]["failed"] and not e["mlp"]["failed"]]
    if ok:
        rw = np.array([e["mlp"]["work"] / e["heuristic"]["work"] for e in ok])
        rt = np.array([e["mlp"]["seconds"] / e["heuristic"]["seconds"] for e in ok])
        s["work_ratio_mlp_over_heuristic"] = {"mean": float(rw.mean()), "median": float(np.median(rw))}
        s["time_ratio_mlp_over_heuristic"] = {"mean": float(rt.mean()), "median": float(np.median(rt))}
    return s


def calibrate_kappa(inst: Instance, n_s: int, factors=(0.5, 0.75, 1.0, 1.5, 2.0, 3.0, 4.0), log=print):
    """kappa = n_p delta~ of the least-work converged run on one instance (the
    heuristic's constant, fixed once and stored with the weights)."""
    H, M = build(inst)
    lo, hi = P.chebfd_bounds(M)
    delta = inst.half_width * 2.0 / (hi - lo)
    runs = []
    for kf in factors:
        n_p = int(round(kf / delta))
        r, dt = run(M, inst, n_p, n_s, max_iter=20)
        w = work_units(M.n, len(H[1]), n_p, n_s, r.stats.iterations)
        log(f"# kappa {kf}: n_p {n_p} status {r.status} iters {r.stats.iterations} found {r.n_found} "
            f"{dt:.2f}s work {w:.3e}")
        runs.append((kf, w, r.status, r.n_found))
    full = max(x[3] for x in runs)
    ok = [x for x in runs if x[2] == 0 and x[3] == full]
    return min(ok, key=lambda x: x[1])[0] if ok else 1.0


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser(description="corpus / training / evaluation of the parameter predictor")
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("corpus")
    c.add_argument("--count", type=int, required=True)
    c.add_argument("--seed", type=int, required=True)
    c.add_argument("--ext", type=int, nargs=2, default=(12, 24))
    c.add_argument("--kappa", type=float, required=True)
    c.add_argument("--counts", type=float, nargs=2, default=None,
                   help="size each interval for an eigenvalue count drawn from this range")
    c.add_argument("--adaptive", action="store_true",
                   help="label by doubling n_p from the heuristic's until pairs are found")
    c.add_argument("--start-np", type=int, default=50, help="adaptive labels start at max(heuristic, this)")
    c.add_argument("--out", required=True)
    k = sub.add_parser("kappa")
    k.add_argument("--dims", type=int, nargs=3, default=(16, 16, 8))
    t = sub.add_parser("train")
    t.add_argument("--corpus", nargs="+", required=True)
    t.add_argument("--kappa", type=float, default=None,
                   help="heuristic constant stored with the weights (default: median n_p delta~ of the labels)")
    t.add_argument("--steps", type=int, default=3000)
    t.add_argument("--out", default=DEFAULT_WEIGHTS)
    e = sub.add_parser("eval")
    e.add_argument("--corpus", nargs="+", required=True)
    e.add_argument("--weights", default=DEFAULT_WEIGHTS)
    e.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    assert torch.cuda.is_available(), "the predictor runs on the GPU"
    P.load()
    log = lambda s: print(s, flush=True)  # noqa: E731
    if a.cmd == "kappa":
        inst = Instance(dims=tuple(a.dims), m=1.0, W=1.0, half_width=0.05, seed=1001)
        log(json.dumps({"kappa": calibrate_kappa(inst, 32, log=log)}))
    elif a.cmd == "corpus":
        make_corpus(a.count, a.seed, a.ext[0], a.ext[1], a.kappa,
                    count_range=None if a.counts is None else tuple(a.counts), log=log,
                    adaptive=a.adaptive, start_np=a.start_np, out=a.out)
    elif a.cmd == "train":
        rows = [r for p in a.corpus for r in json.load(open(p)) if r["label"] is not None and r["full_count"] > 0]
        X = np.array([features_of(r) for r in rows], dtype=np.float32)
        T, mean, std = standardise(targets(rows))
        t_lo, t_hi = target_range(targets(rows))
        kappa = kappa_from_corpus(rows) if a.kappa is None else a.kappa
        params = train(X, T, steps=a.steps, log=log)
        save(a.out, params, mean, std, kappa, {"train_instances": len(rows), "steps": a.steps,
                                               "targets": "log(n_p delta), log(n_s / max(2 n_hat, n_b))",
                                               "corpus": [os.path.basename(p) for p in a.corpus]},
             t_lo=t_lo, t_hi=t_hi)
        log(f"# kappa {kappa:.3f}")
        log(f"# saved {a.out}")
    elif a.cmd == "eval":
        rows = [r for p in a.corpus for r in json.load(open(p))]
        pred = load(a.weights)
        ev = evaluate(pred, rows, pred["kappa"], log=log)
        summ = summarise(ev)
        with open(a.out, "w") as f:
            json.dump({"summary": summ, "runs": ev}, f, indent=1)
        log(json.dumps(summ))


if __name__ == "__main__":
    main()
