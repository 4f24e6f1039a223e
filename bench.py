"""Benchmark of the octree-scoped free-mesh interpolant on one MI355X.

One step = the whole hot path on one batch of synthetic input: fit N points
(keys, sort, gather, per-level Gram / solve / refinement / residual /
topology) and evaluate the fresh tree at Nq queries.  Default workload: N = 2^20
uniform points in the unit cube (float32 storage), values from a seeded sum of
four anisotropic Gaussian bumps, p = 6 (calL = 84), depth <= 6, tol 1e-8,
Nq = 2^22 uniform queries.  Inputs are device-resident before timing starts.

Prints one JSON line (rank 0).  `value` is fit points/s of the headline path;
eval points/s, both paths' errors against the true function, step latency
percentiles, the roofline of the dominant kernel and the CPU oracle baseline
ride along in the same line.
"""
import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3}


def gram_flops_per_point(L: int) -> float:
    # symmetric Gram L(L+1) + right-hand side 2L + basis generation L
    return L * (L + 1) + 2 * L + L


def basis_count(p: int) -> int:
    return (p + 1) * (p + 2) * (p + 3) // 6


def moment_flops_per_point(p: int) -> float:
    # one multiply-add per power moment (|gamma| <= 2p), per r-weighted moment
    # (|alpha| <= p) and for r^2, one product u^a v^b per run, and the powers
    nm, nb = basis_count(2 * p), basis_count(p)
    runs = (2 * p + 1) * (2 * p + 2) // 2 + (p + 1) * (p + 2) // 2
    return 2.0 * (nm + nb + 1) + runs + 3 * 2 * p


def bmoment_flops_per_point(p: int) -> float:
    # r-weighted moments only (|alpha| <= p): one multiply-add each, one
    # product per run, and the powers up to p
    return 2.0 * basis_count(p) + (p + 1) * (p + 2) // 2 + 3 * p


def base_moment_flops_per_point(p: int) -> float:
    # power moments only (|gamma| <= 2p), once per point at the pyramid's
    # finest level
    return 2.0 * basis_count(2 * p) + (2 * p + 1) * (2 * p + 2) // 2 + 3 * 2 * p


def refine_flops_per_point(p: int) -> float:
    # r' = r - Lambda F (about 2L) and the r'-weighted moments (2L + runs + powers)
    L = basis_count(p)
    return 2.0 * L + 2.0 * L + (p + 1) * (p + 2) // 2 + 3 * 2 * p


def solve_flops_per_node(L: int) -> float:
    # Cholesky L^3/3 + forward and back substitution 2L^2
    return L ** 3 / 3.0 + 2.0 * L * L


def eval_flops_per_query(L: int) -> float:
    # one multiply-add per coefficient of the node's composite polynomial
    return 2.0 * L


def kernel_rooflines(kern: dict, p: int, L: int, path: str, coord_bytes: int, steps: int, key_passes: int,
                     eval_key_passes: int):
    """Achieved rate of each kernel class over the timed steps: algorithmic work
    (flops or bytes per unit times the units the launches covered) divided by
    the summed launch durations measured with HIP events."""
    out = {}
    def add(name, bound, per_unit, unit, peak):
        st = kern.get(name)
        if not st or st["ms_per_step"] <= 0:
            return
        sec = st["ms_per_step"] * steps / 1e3
        work = st["units"] * per_unit
        scale = 1e12 if unit == "TFLOP/s" else 1e9
        ach = work / sec / scale
        out[name] = dict(bound=bound, achieved=ach, peak=peak, unit=unit, frac=ach / peak,
                         avg_launch_ms=st["avg_launch_ms"], work_per_unit=per_unit,
                         units_per_step=st["units"] / steps)
    if path == "mixed":
        add("gram", "mfma", gram_flops_per_point(L), "TFLOP/s", PEAK_TFLOPS["fp32"])
    else:
        add("gram", "alu", moment_flops_per_point(p), "TFLOP/s", PEAK_TFLOPS["fp64"])
    add("bmoments", "alu", bmoment_flops_per_point(p), "TFLOP/s", PEAK_TFLOPS["fp64"])
    add("base_moments", "alu", base_moment_flops_per_point(p), "TFLOP/s", PEAK_TFLOPS["fp64"])
    add("solve", "alu", solve_flops_per_node(L), "TFLOP/s", PEAK_TFLOPS["fp64"])
    # the pyramid's upper levels: factors made ahead of the level loop (units:
    # cells), then per level only the two triangular solves (units: nodes)
    add("factor_ahead", "alu", L ** 3 / 3.0, "TFLOP/s", PEAK_TFLOPS["fp64"])
    add("solve_ahead", "alu", 2.0 * L * L, "TFLOP/s", PEAK_TFLOPS["fp64"])
    if path == "mixed":
        # every node is refined; on the float64 path only the nodes the
        # condition estimate flags are, a count the host does not see, so the
        # launches' units (all of the level's points and nodes) would overstate
        # the work
        add("refine_solve", "alu", 2.0 * L * L, "TFLOP/s", PEAK_TFLOPS["fp64"])
        add("refine_sweep", "alu", refine_flops_per_point(p), "TFLOP/s", PEAK_TFLOPS["fp64"])
    # residual: coordinates + residual read, residual written, key read
    add("residual", "hbm", 3 * coord_bytes + 8 + 8 + 4, "GB/s", PEAK_HBM_GBS)
    # sort: per pass read and write key and index, and the payload (the fit
    # moves x, y, z, f; the evaluation x, y, z), plus the histogram's key read
    add("sort", "hbm", (20.0 + 8 * coord_bytes) * key_passes, "GB/s", PEAK_HBM_GBS)
    add("eval_sort", "hbm", (20.0 + 6 * coord_bytes) * eval_key_passes, "GB/s", PEAK_HBM_GBS)
    # residual start: sorted values in, float64 residual out
    add("gather", "hbm", coord_bytes + 8, "GB/s", PEAK_HBM_GBS)
    # query keys: coordinates in, key out
    add("eval_keys", "hbm", 3 * coord_bytes + 4, "GB/s", PEAK_HBM_GBS)
    # evaluation: the bound is whichever of its flops (2L per query) and its
    # bytes (coordinates in, value out) takes longer at peak
    t_flop = eval_flops_per_query(L) / (PEAK_TFLOPS["fp64"] * 1e12)
    t_byte = (3 * coord_bytes + 8) / (PEAK_HBM_GBS * 1e9)
    if t_flop >= t_byte:
        add("eval", "alu", eval_flops_per_query(L), "TFLOP/s", PEAK_TFLOPS["fp64"])
    else:
        add("eval", "hbm", 3 * coord_bytes + 8, "GB/s", PEAK_HBM_GBS)
    # chunk reduction: units are partial doubles read (the result writes are
    # one chunk's worth per node)
    add("gram_reduce", "hbm", 8.0, "GB/s", PEAK_HBM_GBS)
    # child activation: 16 partial doubles in, 8 begins + 8 counts + mask +
    # active count out, begin read, per node
    add("children", "hbm", 16 * 8 + 16 * 4 + 12, "GB/s", PEAK_HBM_GBS)
    return out


def refit_rooflines(kern: dict, p: int, L: int, coord_bytes: int, steps: int, fields: int = 1):
    """Rooflines of the fixed-topology refit's kernel classes (same definition
    as kernel_rooflines: algorithmic work over summed launch durations)."""
    out = {}
    def add(name, bound, per_unit, unit, peak):
        st = kern.get(name)
        if not st or st["ms_per_step"] <= 0:
            return
        sec = st["ms_per_step"] * steps / 1e3
        scale = 1e12 if unit == "TFLOP/s" else 1e9
        ach = st["units"] * per_unit / sec / scale
        out[name] = dict(bound=bound, achieved=ach, peak=peak, unit=unit, frac=ach / peak,
                         avg_launch_ms=st["avg_launch_ms"], work_per_unit=per_unit,
                         units_per_step=st["units"] / steps, traffic=None)
    # power moments M: from the moment pyramid (one pass over the points) for
    # the levels it covers, else once per level (mode 3); the factor once per
    # node
    add("base_moments", "alu", base_moment_flops_per_point(p), "TFLOP/s", PEAK_TFLOPS["fp64"])
    add("refit_moments", "alu", base_moment_flops_per_point(p), "TFLOP/s", PEAK_TFLOPS["fp64"])
    add("refit_factor", "alu", L ** 3 / 3.0, "TFLOP/s", PEAK_TFLOPS["fp64"])
    # per field: B (mode 2), two triangular solves, the residual update
    add("refit_bmoments", "alu", bmoment_flops_per_point(p), "TFLOP/s", PEAK_TFLOPS["fp64"])
    add("refit_solve", "alu", 2.0 * L * L, "TFLOP/s", PEAK_TFLOPS["fp64"])
    # residual: r read and written per field, the coordinates once per point
    # for all the fields
    add("refit_residual", "hbm", 8 + 8 + 3 * coord_bytes / max(fields, 1), "GB/s", PEAK_HBM_GBS)
    return out


def refit_leg(fmt, tree_opts, X, Y, Z, pr, m: int, steps: int, warmup: int):
    """Fixed-topology refit of m new fields on the headline tree: wall time
    per call (inputs resident, the call returns with the trees complete) and
    per-kernel launch durations in a second, profiled pass."""
    import numpy as np
    import torch

    import synthetic
    fields = np.stack([synthetic.bumps_value(synthetic.draw_bumps(900 + j), pr.x, pr.y, pr.z).astype(pr.x.dtype)
                       for j in range(m)])
    FF = torch.from_numpy(fields).cuda()
    tree = fmt.fmt_fit(tree_opts, X, Y, Z, torch.from_numpy(np.ascontiguousarray(pr.f)).cuda())
    for _ in range(warmup):
        for t in fmt.fmt_refit(tree, X, Y, Z, FF):
            t.close()
    torch.cuda.synchronize()
    times = []
    for _ in range(steps):
        t0 = time.perf_counter()
        outs = fmt.fmt_refit(tree, X, Y, Z, FF)
        times.append(time.perf_counter() - t0)
        for t in outs:
            t.close()
    fmt.fmt_profile_reset()
    fmt.fmt_profile_enable(True)
    for _ in range(steps):
        for t in fmt.fmt_refit(tree, X, Y, Z, FF):
            t.close()
    torch.cuda.synchronize()
    fmt.fmt_profile_enable(False)
    prof = fmt.fmt_profile_read()
    nodes = int(tree.info().nodes)
    tree.close()
    kern = {k: dict(launches=v[0], ms_per_step=v[1] / steps, avg_launch_ms=(v[1] / v[0] if v[0] else 0.0),
                    units=v[2]) for k, v in prof.items() if v[0]}
    L = basis_count(pr.p)
    t50 = statistics.median(times)
    return {
        "fields": m, "n": pr.n, "nodes": nodes,
        "ms_p50": 1e3 * t50, "ms_p99": 1e3 * float(np.percentile(times, 99)),
        "field_pts_per_s": m * pr.n / t50,
        "rooflines": refit_rooflines(kern, pr.p, L, pr.x.dtype.itemsize, steps, m),
        "kernels": {k: {kk: round(vv, 6) if isinstance(vv, float) else vv for kk, vv in st.items()}
                    for k, st in kern.items()},
    }


def _progress(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def batched_leg(fmt, steps: int, warmup: int):
    """Batched workload: 256 independent fits of uneven size (N log-uniform in
    [1e3, 2e5], Gaussian-mixture points, p in {4, 5, 6}) in one fmt_fit_batch
    call, each problem's 4 096 mixture queries evaluated; the mixed path (the
    workload's float32 Gram + float64 solve) and the float64 path."""
    import numpy as np
    import torch

    import synthetic
    probs = synthetic.config3()
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    X = [dev(pr.x) for pr in probs]
    Y = [dev(pr.y) for pr in probs]
    Z = [dev(pr.z) for pr in probs]
    Fv = [dev(pr.f) for pr in probs]
    Q = [(dev(pr.qx), dev(pr.qy), dev(pr.qz)) for pr in probs]
    outs = [torch.empty(pr.qx.shape[0], dtype=torch.float64, device="cuda") for pr in probs]
    total = sum(pr.n for pr in probs)
    nq = sum(pr.qx.shape[0] for pr in probs)
    truth = np.concatenate([pr.qf_true for pr in probs])
    res = {}
    for path in ("mixed", "fp64"):
        opts = [fmt.fmt_default_opts(p=pr.p, tol=pr.tol, max_depth=pr.max_depth, refine_steps=1,
                                     path=fmt.FMT_PATH_MIXED if path == "mixed" else fmt.FMT_PATH_FP64)
                for pr in probs]
        for _ in range(max(1, warmup)):
            for t in fmt.fmt_fit_batch(opts, X, Y, Z, Fv):
                t.close()
        torch.cuda.synchronize()
        fit_t, eval_t = [], []
        for _ in range(steps):
            t0 = time.perf_counter()
            trees = fmt.fmt_fit_batch(opts, X, Y, Z, Fv)   # returns with every tree complete
            t1 = time.perf_counter()
            for tr, (qx, qy, qz), o in zip(trees, Q, outs):
                tr.eval(qx, qy, qz, out=o)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            fit_t.append(t1 - t0)
            eval_t.append(t2 - t1)
            nodes = sum(int(t.info().nodes) for t in trees)
            for t in trees:
                t.close()
        got = np.concatenate([o.cpu().numpy() for o in outs])
        res[path] = {"fit_pts_per_s": total / statistics.median(fit_t),
                     "fit_ms_p50": 1e3 * statistics.median(fit_t), "fit_ms_p99": 1e3 * float(np.percentile(fit_t, 99)),
                     "eval_pts_per_s": nq / statistics.median(eval_t),
                     "eval_ms_p50": 1e3 * statistics.median(eval_t), "nodes": nodes,
                     "E_rms": float(np.sqrt(np.mean((got - truth) ** 2)))}
        _progress(f"batched {path}: {res[path]['fit_ms_p50']:.2f} ms per batch")
    return {"workload": "batched uneven problems: 256 fits in one fmt_fit_batch call, N log-uniform [1e3, 2e5] "
                        "(float32 Gaussian-mixture points, 1-8 components), p in {4,5,6}, depth<=6, tol 1e-8; "
                        "4096 mixture queries per problem",
            "problems": len(probs), "points": total, "queries": nq,
            "value": res["mixed"]["fit_pts_per_s"], "unit": "fit points/s (mixed path)",
            "paths": res,
            "E_rms_ratio_minus_1": res["mixed"]["E_rms"] / res["fp64"]["E_rms"] - 1.0}


def served_leg():
    """Served workload: continuous batching of a Poisson request stream (the
    serve module), latency percentiles at 50% and 80% of the measured
    saturation rate, device memory against the budget."""
    from paper_1511_01353_amd.serve import serve_report
    rep = serve_report(requests=120, budget_gb=16.0, streams=4, seed=4000, loads=(0.5, 0.8), fit_slots=2,
                       progress=_progress)
    rep["note"] = "request payloads are host arrays, so latencies include their host-to-device copies"
    return rep


def clustered_leg(fmt, steps: int, warmup: int):
    """Large clustered workload: 2^26 float32 points from a 32-component
    Gaussian mixture, p = 8, depth <= 10, tol 1e-8; 2^26 mixture queries
    (sorted evaluation: the coefficient table is tens of MB); the mixed path
    (the workload's float32 MFMA Gram + float64 solve + one refinement sweep)
    and the float64 path; errors against the true function and, when the
    stored oracle values are present, against the oracle on its sample."""
    import numpy as np
    import torch

    import synthetic
    t0 = time.perf_counter()
    pr = synthetic.config5()
    _progress(f"clustered inputs in {time.perf_counter() - t0:.0f} s")
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    X, Y, Z, Fv = dev(pr.x), dev(pr.y), dev(pr.z), dev(pr.f)
    QX, QY, QZ = dev(pr.qx), dev(pr.qy), dev(pr.qz)
    out = torch.empty(QX.numel(), dtype=torch.float64, device="cuda")
    gold = None
    gpath = os.path.join(ROOT, "tests", "golden", "config5_oracle.npz")
    if os.path.exists(gpath):
        gold = np.load(gpath)
    res = {}
    for path in ("mixed", "fp64"):
        opts = fmt.fmt_default_opts(p=pr.p, tol=pr.tol, max_depth=pr.max_depth, refine_steps=1,
                                    path=fmt.FMT_PATH_MIXED if path == "mixed" else fmt.FMT_PATH_FP64)
        for _ in range(max(1, warmup)):
            t = fmt.fmt_fit(opts, X, Y, Z, Fv)
            t.eval(QX, QY, QZ, out=out, sort_queries=1)
            t.close()
        torch.cuda.synchronize()
        fit_t, eval_t = [], []
        for k in range(steps):
            t0 = time.perf_counter()
            tree = fmt.fmt_fit(opts, X, Y, Z, Fv)
            t1 = time.perf_counter()
            tree.eval(QX, QY, QZ, out=out, sort_queries=1)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            fit_t.append(t1 - t0)
            eval_t.append(t2 - t1)
            if k + 1 < steps:
                tree.close()
        fq = out.cpu().numpy()
        info = tree.info()
        r = {"fit_pts_per_s": pr.n / statistics.median(fit_t), "fit_ms_p50": 1e3 * statistics.median(fit_t),
             "eval_pts_per_s": QX.numel() / statistics.median(eval_t), "eval_ms_p50": 1e3 * statistics.median(eval_t),
             "nodes": int(info.nodes), "depth": int(info.depth),
             "E_rms": float(np.sqrt(np.mean((fq - pr.qf_true) ** 2))), "E_inf": float(np.max(np.abs(fq - pr.qf_true)))}
        if gold is not None:
            sel = gold["query_index"]
            ok = (~gold["rank"]) & (gold["kappa"] <= 1e8) & (gold["h"] <= 1e4)
            d = (fq[sel] - gold["want"]) / np.maximum(1.0, np.sqrt(np.where(ok, gold["h"], 0.0)))
            pts = tree.export_points()
            r["vs_oracle"] = {"queries_compared": int(ok.sum()), "of": int(sel.shape[0]),
                              "eval_rms_scaled_diff": float(np.sqrt(np.mean(d[ok] ** 2))),
                              "residual_rms_diff": float(np.sqrt(np.mean(
                                  (pts["residual"][gold["point_index"]] - gold["residual"]) ** 2)))}
        tree.close()
        res[path] = r
        _progress(f"clustered {path}: fit {r['fit_ms_p50']:.1f} ms, eval {r['eval_ms_p50']:.1f} ms")
    return {"workload": "large clustered fit: N=2^26 float32 points from a 32-component Gaussian mixture, "
                        "4 Gaussian bumps, p=8 (L=165), depth<=10, tol 1e-8; eval 2^26 mixture queries, sorted",
            "value": res["mixed"]["fit_pts_per_s"], "unit": "fit points/s (mixed path)",
            "paths": res, "E_rms_ratio_minus_1": res["mixed"]["E_rms"] / res["fp64"]["E_rms"] - 1.0,
            "oracle_fit_seconds": float(gold["fit_seconds"]) if gold is not None else None,
            "oracle_threads": int(gold["threads"]) if gold is not None else None}


def rbf_leg(fmt, steps: int):
    """Gaussian-RBF factorisation check: 16384 query points against 16384
    points in [-1, 1]^3 (float64), eps = 0.15, orders 6, 10 and 14; launch
    times of the two MFMA products from HIP events; the largest deviation from
    the directly evaluated Gaussian on a 256 x 256 corner of the block."""
    import numpy as np
    import torch
    n = nq = 1 << 14
    rng = np.random.default_rng(8000)
    x = [torch.from_numpy(a).cuda() for a in rng.uniform(-1.0, 1.0, (3, n))]
    q = [torch.from_numpy(a).cuda() for a in rng.uniform(-1.0, 1.0, (3, nq))]
    out = torch.empty((nq, n), dtype=torch.float64, device="cuda")
    eps = 0.15
    res = {}
    for p in (6, 10, 14):
        L = basis_count(p)
        fmt.fmt_rbf_factored(p, eps, *x, *q, out=out)
        torch.cuda.synchronize()
        fmt.fmt_profile_reset()
        fmt.fmt_profile_enable(True)
        t0 = time.perf_counter()
        for _ in range(steps):
            fmt.fmt_rbf_factored(p, eps, *x, *q, out=out)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / steps
        fmt.fmt_profile_enable(False)
        prof = fmt.fmt_profile_read()
        pairs = prof.get("rbf_pairs", (0, 0.0, 0.0))
        ms = pairs[1] / max(pairs[0], 1)
        flops = 2.0 * n * nq * L
        xs = [a[:256].cpu().numpy() for a in x]
        qs = [a[:256].cpu().numpy() for a in q]
        d2 = sum((qa[:, None] - xa[None, :]) ** 2 for qa, xa in zip(qs, xs))
        dev = float(np.max(np.abs(out[:256, :256].cpu().numpy() - np.exp(-eps * eps * d2))))
        res[f"p{p}"] = {"calL": L, "pairs_ms": ms, "wall_ms": 1e3 * wall,
                        "roofline": {"bound": "mfma", "achieved": flops / (ms * 1e-3) / 1e12,
                                     "peak": PEAK_TFLOPS["fp64"], "unit": "TFLOP/s",
                                     "frac": flops / (ms * 1e-3) / 1e12 / PEAK_TFLOPS["fp64"]},
                        "max_dev_from_gaussian": dev}
        _progress(f"rbf p={p}: {ms:.2f} ms, {res[f'p{p}']['roofline']['frac']:.3f} of the fp64 MFMA peak")
    return {"workload": "Gaussian-RBF factorisation check: 16384 x 16384 float64 block, points and queries "
                        "uniform in [-1,1]^3, eps 0.15, orders 6/10/14",
            "work_per_unit": "2 calL flops per (query, point) pair", "paths": res}


def wide_leg(fmt, steps: int):
    """Large bases: the unscoped single-node fits of Section 3 (8^6 uniform
    points of the Franke function, depth 0) at orders 10 and 14, and the
    scoped order-12 fit of Section 4 at 8^7 points, tol 1e-10."""
    import numpy as np
    import torch

    import synthetic
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    res = {}
    for name, n, p, tol, depth in (("unscoped_p10", 8 ** 6, 10, 0.0, 0), ("unscoped_p14", 8 ** 6, 14, 0.0, 0),
                                   ("scoped_p12", 8 ** 7, 12, 1e-10, 10)):
        pr = synthetic.scoping_problem(n, p, tol, 6300, depth=depth)
        X = [dev(a) for a in (pr.x, pr.y, pr.z, pr.f)]
        Q = [dev(a) for a in (pr.qx, pr.qy, pr.qz)]
        o = fmt.fmt_default_opts(p=p, tol=tol, max_depth=depth)
        fmt.fmt_fit(o, *X).close()
        torch.cuda.synchronize()
        ts = []
        for k in range(steps):
            t0 = time.perf_counter()
            tr = fmt.fmt_fit(o, *X)
            ts.append(time.perf_counter() - t0)
            if k + 1 < steps:
                tr.close()
        got = tr.eval(*Q).cpu().numpy()
        err = got - pr.qf_true
        res[name] = {"n": n, "p": p, "calL": basis_count(p), "tol": tol, "nodes": int(tr.info().nodes),
                     "fit_ms_p50": 1e3 * statistics.median(ts), "fit_pts_per_s": n / statistics.median(ts),
                     "E_rms": float(np.sqrt(np.mean(err * err))), "E_inf": float(np.max(np.abs(err)))}
        tr.close()
        _progress(f"wide {name}: {res[name]['fit_ms_p50']:.1f} ms")
    return {"workload": "large bases: unscoped 8^6-point Franke fits at p=10, 14; scoped 8^7-point fit at p=12, "
                        "tol 1e-10 (float64 path)", "cases": res}


def kernel_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    src = os.path.join(ROOT, "paper_1511_01353_amd", "csrc")
    for f in sorted(os.listdir(src)):
        if f.endswith(".hip") or f.endswith(".h"):
            h.update(f.encode())
            with open(os.path.join(src, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """Per-class HBM bytes per launch from the committed rocprofv3 --pmc summary,
    or None when the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_fit_eval_n2p20_p6.md")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        text = fh.read()
    tag = "<!-- traffic-json: "
    if tag not in text:
        return None
    doc = json.loads(text.split(tag, 1)[1].split(" -->", 1)[0])
    if doc.get("sources_sha256") != kernel_sources_sha256():
        return None
    return {c: v["fetch_bytes_per_launch"] + v["write_bytes_per_launch"] for c, v in doc["classes"].items()}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--path", choices=["fp64", "mixed"], default="fp64", help="headline path")
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--nq", type=int, default=1 << 22)
    ap.add_argument("--sort-queries", type=int, default=-1)
    ap.add_argument("--mixed-refine", type=int, default=1)
    ap.add_argument("--fp64-refine", type=int, default=1)
    ap.add_argument("--no-compare", action="store_true", help="time only the headline path")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1 << 16,
                    help="points of the benchmark workload the one-thread oracle baseline fits")
    ap.add_argument("--configs", type=str, default="3,4,5,wide,rbf",
                    help="other workloads to run after the headline: 3 batched, 4 served, 5 large clustered, "
                         "wide (large bases), rbf (the Gaussian-RBF factorisation check)")
    ap.add_argument("--refit-fields", type=int, default=8,
                    help="value fields of the fixed-topology refit leg (0: skip it)")
    ap.add_argument("--refit-only", action="store_true",
                    help="run only the refit leg and print its object (for profiling it alone)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="after the run, copy this many MiB device to device (a plain copy kernel of known size "
                         "against which hardware byte counters are scaled)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU; --gpus N with N > 1 is not supported", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1511_01353_amd as fmt
    import synthetic

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    fmt.load_library()
    torch.cuda.set_device(0)
    pr = synthetic.config2(n=args.n, nq=args.nq)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    X, Y, Z, Fv = dev(pr.x), dev(pr.y), dev(pr.z), dev(pr.f)
    QX, QY, QZ = dev(pr.qx), dev(pr.qy), dev(pr.qz)
    out = torch.empty(args.nq, dtype=torch.float64, device="cuda")
    L = (pr.p + 1) * (pr.p + 2) * (pr.p + 3) // 6
    if args.refit_only:
        opts = fmt.fmt_default_opts(p=pr.p, tol=pr.tol, max_depth=pr.max_depth, refine_steps=args.fp64_refine)
        print(json.dumps({"refit": refit_leg(fmt, opts, X, Y, Z, pr, max(1, args.refit_fields), args.steps,
                                             args.warmup)}))
        return
    paths = [args.path] if args.no_compare else [args.path] + [p for p in ("fp64", "mixed") if p != args.path]
    results = {}
    kept = {}
    for path in paths:
        opts = fmt.fmt_default_opts(p=pr.p, tol=pr.tol, max_depth=pr.max_depth,
                                    path=fmt.FMT_PATH_MIXED if path == "mixed" else fmt.FMT_PATH_FP64,
                                    refine_steps=args.mixed_refine if path == "mixed" else args.fp64_refine)

        def step():
            t0 = time.perf_counter()
            tree = fmt.fmt_fit(opts, X, Y, Z, Fv)          # returns with the tree complete
            t1 = time.perf_counter()
            tree.eval(QX, QY, QZ, out=out, sort_queries=args.sort_queries)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            return tree, t1 - t0, t2 - t1

        for _ in range(args.warmup):
            tree, _, _ = step()
            tree.close()
        timed = path == args.path
        torch.cuda.synchronize()
        fit_t, eval_t = [], []
        T0 = time.perf_counter()
        for _ in range(args.steps):
            tree, a, b = step()
            fit_t.append(a)
            eval_t.append(b)
            if _ + 1 < args.steps:
                tree.close()
            last = tree
        torch.cuda.synchronize()
        T1 = time.perf_counter()
        # per-kernel launch durations: HIP events around every launch, in a
        # second pass of the same steps (kept out of the timed pass above)
        fmt.fmt_profile_reset()
        fmt.fmt_profile_enable(True)
        for _ in range(args.steps):
            tree, _, _ = step()
            tree.close()
        torch.cuda.synchronize()
        fmt.fmt_profile_enable(False)
        prof = fmt.fmt_profile_read()
        info = last.info()
        fq = out.cpu().numpy()
        e_rms = float(np.sqrt(np.mean((fq - pr.qf_true) ** 2)))
        e_inf = float(np.max(np.abs(fq - pr.qf_true)))
        # kept for the comparison with the oracle's fit of the same workload
        kept[path] = dict(residual=last.export_points()["residual"], nodes=last.export_nodes(), fq=fq)
        last.close()
        results[path] = dict(
            fit_pts_per_s=args.n * len(fit_t) / sum(fit_t),
            eval_pts_per_s=args.nq * len(eval_t) / sum(eval_t),
            fit_ms_p50=1e3 * statistics.median(fit_t),
            fit_ms_p99=1e3 * float(np.percentile(fit_t, 99)),
            eval_ms_p50=1e3 * statistics.median(eval_t),
            eval_ms_p99=1e3 * float(np.percentile(eval_t, 99)),
            step_ms=1e3 * (T1 - T0) / args.steps,
            E_rms=e_rms, E_inf=e_inf, nodes=int(info.nodes),
            per_level=[int(info.per_level[i]) for i in range(info.depth + 1)],
            kernels={k: dict(launches=v[0], ms_per_step=v[1] / args.steps,
                             avg_launch_ms=(v[1] / v[0] if v[0] else 0.0), units=v[2])
                     for k, v in prof.items() if v[0]},
        )
        if timed:
            headline = results[path]
            headline["wall_s"] = T1 - T0

    h = results[args.path]
    key_passes = max(1, (3 * pr.max_depth + 7) // 8)
    eval_key_passes = max(1, (3 * (len(h["per_level"]) - 1) + 7) // 8)
    roofs = kernel_rooflines(h["kernels"], pr.p, L, args.path, pr.x.dtype.itemsize, args.steps, key_passes,
                             eval_key_passes)
    # the dominant kernel of the headline path's step (by time) among those
    # with a roofline definition
    dom = max((kv for kv in h["kernels"].items() if kv[0] in roofs), key=lambda kv: kv[1]["ms_per_step"])[0]
    roof = dict(kernel=dom, **roofs[dom])
    traffic = measured_traffic() if args.path == "fp64" and args.n == 1 << 20 and args.nq == 1 << 22 else None
    roof["traffic"] = traffic.get(dom) if traffic else None
    for k, v in roofs.items():
        v["traffic"] = traffic.get(k) if traffic else None
    gram_roof = roofs.get("gram")

    refit = None
    if args.refit_fields > 0:
        opts = fmt.fmt_default_opts(p=pr.p, tol=pr.tol, max_depth=pr.max_depth,
                                    path=fmt.FMT_PATH_MIXED if args.path == "mixed" else fmt.FMT_PATH_FP64,
                                    refine_steps=args.mixed_refine if args.path == "mixed" else args.fp64_refine)
        refit = refit_leg(fmt, opts, X, Y, Z, pr, args.refit_fields, args.steps, args.warmup)

    others = {}
    want = {c.strip() for c in args.configs.split(",") if c.strip()}
    if "3" in want:
        others["cfg3"] = batched_leg(fmt, max(3, args.steps // 2), 1)
    if "4" in want:
        others["cfg4"] = served_leg()
    if "5" in want:
        others["cfg5"] = clustered_leg(fmt, 3, 1)
    if "wide" in want:
        others["large_bases"] = wide_leg(fmt, 3)
    if "rbf" in want:
        others["rbf_check"] = rbf_leg(fmt, 3)

    cpu = None
    vs_oracle = None
    if not args.no_cpu_baseline:
        cpu, ot = cpu_baseline(pr, args.cpu_sample)
        vs_oracle = oracle_comparison(pr, ot, kept)

    cmp = None
    if "fp64" in results and "mixed" in results:
        cmp = dict(E_rms_ratio_minus_1=results["mixed"]["E_rms"] / results["fp64"]["E_rms"] - 1.0)
    line = {
        "metric": "fit pts/s & eval pts/s at fixed RMS err, mixed vs FP64 GPU; p50/p99 latency",
        "value": h["fit_pts_per_s"],
        "unit": "fit points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h["step_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.path == "fp64" else "f32-mfma+f64",
        "data": "synthetic (seeded uniform points, 4-bump anisotropic Gaussian values)",
        "config": {"workload": "single large fit + eval: N=2^20 uniform fp32 points in [0,1]^3, 4 Gaussian bumps, "
                               "p=6 (L=84), depth<=6, tol=1e-8; eval 2^22 queries",
                   "n": args.n, "nq": args.nq, "p": pr.p, "max_depth": pr.max_depth, "tol": pr.tol,
                   "path": args.path},
        "eval_pts_per_s": h["eval_pts_per_s"],
        "latency_ms": {"fit_p50": h["fit_ms_p50"], "fit_p99": h["fit_ms_p99"], "eval_p50": h["eval_ms_p50"],
                       "eval_p99": h["eval_ms_p99"]},
        "roofline": roof,
        "rooflines": roofs,
        "paths": {k: {kk: vv for kk, vv in v.items() if kk != "kernels"} for k, v in results.items()},
        "kernels": {k: {kk: round(vv, 6) if isinstance(vv, float) else vv for kk, vv in st.items()}
                    for k, st in h["kernels"].items()},
        "mixed_vs_fp64": cmp,
        "vs_oracle": vs_oracle,
        "refit": refit,
        **others,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))
    if args.copy_calibration_mib > 0:
        nb = args.copy_calibration_mib << 20
        src = torch.ones(nb, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nb}), file=sys.stderr)


def cpu_baseline(pr, sample: int):
    """The FP64 oracle on the host cores: the whole benchmark workload on all
    threads (the same tree as the GPU's), a sample of it on one thread, and
    the small workload on one and on all threads."""
    import numpy as np

    import oracle
    import synthetic
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        threadpool_limits = None
        threads = os.cpu_count() or 1

    kept = {}

    def timed(p, n=None):
        n = p.n if n is None else min(n, p.n)
        t0 = time.perf_counter()
        kept["tree"] = oracle.fit(p.x[:n], p.y[:n], p.z[:n], p.f[:n], p.p, p.tol, p.max_depth)
        return n, time.perf_counter() - t0

    n_all, dt_all = timed(pr)
    ot = kept["tree"]
    _progress(f"cpu oracle, {n_all} points, {threads} threads: {dt_all:.1f} s")
    small = synthetic.config1()
    variants = []
    n1, d1 = timed(small)
    variants.append({"workload": "small: N=4096 uniform float64, p=4, depth 3 (73 nodes)", "threads": int(threads),
                     "value": n1 / d1, "seconds": d1})
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            n1, d1 = timed(small)
            variants.append({"workload": "small: N=4096 uniform float64, p=4, depth 3 (73 nodes)", "threads": 1,
                             "value": n1 / d1, "seconds": d1})
            ns, ds = timed(pr, sample)
            variants.append({"workload": f"benchmark workload, first {ns} points", "threads": 1,
                             "value": ns / ds, "seconds": ds})
    return {"value": n_all / dt_all, "unit": "fit points/s", "cores": int(threads), "kind": "oracle",
            "sample": f"all {n_all} points of the benchmark workload (p={pr.p}, depth<={pr.max_depth}, "
                      f"tol={pr.tol}; the same tree as the GPU fit); {dt_all:.1f} s",
            "variants": variants}, ot


def oracle_comparison(pr, ot, kept, nsample: int = 1 << 14):
    """Each path's last fit of the benchmark workload against the oracle's fit
    of the same workload (the baseline leg's): node set, fitted values at the
    points, and evaluation at a seeded sample of the queries."""
    import numpy as np

    import oracle
    sel = np.sort(np.random.default_rng(20).choice(pr.qx.shape[0], nsample, replace=False))
    want = oracle.evaluate(ot, pr.qx[sel], pr.qy[sel], pr.qz[sel])
    out = {}
    for path, k in kept.items():
        nd = k["nodes"]
        same = (nd["level"].shape[0] == ot.nodes and np.array_equal(nd["level"].astype(np.int64), ot.level)
                and np.array_equal(nd["prefix"].astype(np.int64), ot.prefix)
                and np.array_equal(nd["begin"].astype(np.int64), ot.begin)
                and np.array_equal(nd["count"].astype(np.int64), ot.count))
        d = k["fq"][sel] - want
        out[path] = {"nodes_equal": bool(same),
                     "fitted_rms_diff": float(np.sqrt(np.mean((k["residual"] - ot.residual) ** 2))),
                     "eval_rms_diff": float(np.sqrt(np.mean(d ** 2))), "eval_max_diff": float(np.max(np.abs(d))),
                     "queries": int(nsample)}
    return out


if __name__ == "__main__":
    main()
