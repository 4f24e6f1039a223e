"""Continuous-batching request server over the fit / eval C ABI.

Requests arrive over time: a *fit* carries points and values (and fit
options) and produces a tree kept resident in device memory; an *eval*
names a resident tree and carries query points.  The scheduler:

* admits a request only while the device-memory footprint of everything
  admitted and not finished, the resident trees and the library's fit
  workspaces stay under the budget, and only while a slot of its kind is
  free (evals: one per stream of the pool; fits: `fit_slots` batches in
  flight, each on its own stream);
* merges the fits waiting at each tick into one batched fit (one launch per
  level and kernel over all of them), run by a worker thread on a fit
  stream, so fits overlap on the device with other fit batches and with
  evaluations launched meanwhile on the eval streams;
* evicts least-recently-used resident trees to make room for new work;
* records, per request, arrival -> admission -> completion times, from which
  p50 / p99 latency and throughput follow, and samples the device memory
  actually in use (when the executor can measure it) against the budget.

The device work goes through an ``Executor``; ``GpuExecutor`` drives the
library, and tests drive the scheduler with a scripted fake executor.
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time
from typing import Callable, Dict, List, Optional

import numpy as np

__all__ = ["Request", "Server", "GpuExecutor", "fit_footprint", "eval_footprint", "tree_footprint",
           "percentile"]


# ----------------------------------------------------------------------------
# footprints (bytes of device memory a request holds while it runs)
# ----------------------------------------------------------------------------
def fit_footprint(n: int, p: int, itemsize: int = 4) -> int:
    # inputs (x, y, z, f), sorted copies, residual, keys/order (+ sort buffers),
    # level scratch and the worst-case node table
    L = (p + 1) * (p + 2) * (p + 3) // 6
    per_point = 4 * itemsize + 3 * itemsize + 8 + 4 * 4 + 64
    nodes = max(1, n // L) * 2
    return int(n * per_point + nodes * (8 * L + 96) + (1 << 20))


def tree_footprint(n: int, p: int) -> int:
    L = (p + 1) * (p + 2) * (p + 3) // 6
    nodes = max(1, n // L) * 2
    return int(n * 16 + nodes * (8 * L + 96))


def workspace_footprint(n: int, p: int, itemsize: int = 4) -> int:
    # the library's per-stream fit workspace grows to the largest fit run on
    # the stream and stays: two sets of sorted inputs, key/index buffers,
    # sort histograms, moment partials and the pyramid of the top levels
    L = (p + 1) * (p + 2) * (p + 3) // 6
    M = (2 * p + 1) * (2 * p + 2) * (2 * p + 3) // 6
    return int(n * (8 * itemsize + 16) + (n // 2048 + 4096) * 8 * (M + L + 17) + (64 << 20))


def eval_footprint(nq: int, itemsize: int = 4) -> int:
    # queries, output, sort keys/indices and permuted queries
    return int(nq * (3 * itemsize + 8 + 16 + 3 * itemsize) + (1 << 20))


def percentile(xs: List[float], q: float) -> float:
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q)) if xs else float("nan")


# ----------------------------------------------------------------------------
# requests
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Request:
    rid: int
    kind: str                      # "fit" or "eval"
    arrival: float                 # seconds, on the server clock
    n: int                         # points (fit) or queries (eval)
    payload: object = None         # executor-specific inputs
    tree: Optional[int] = None     # eval: rid of the fit whose tree it uses
    opts: dict = dataclasses.field(default_factory=dict)
    footprint: int = 0
    admitted: float = float("nan")
    done: float = float("nan")
    result: object = None
    error: Optional[str] = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


# ----------------------------------------------------------------------------
# the scheduler
# ----------------------------------------------------------------------------
class Server:
    def __init__(self, executor, budget_bytes: int, eval_slots: int = 4, clock: Callable[[], float] = None,
                 fit_slots: int = 2):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.eval_slots = int(eval_slots)
        self.fit_slots = max(1, int(fit_slots))
        self.clock = clock or time.perf_counter
        self.t0 = self.clock()
        self.pending: collections.deque = collections.deque()
        self.running_evals: List[tuple] = []          # (request, handle)
        self.running_fits: List[tuple] = []            # (requests, handle, slot)
        self.ws = [0] * self.fit_slots                 # workspace high-water of each fit stream
        self.trees: "collections.OrderedDict[int, tuple]" = collections.OrderedDict()  # rid -> (tree, bytes)
        self.in_use = 0                                # bytes of running requests
        self.peak = 0
        self.peak_measured = None                      # bytes, if the executor measures device memory
        self.finished: List[Request] = []
        self.deferred = 0
        self.evicted: set = set()

    # --- bookkeeping -------------------------------------------------------
    def now(self) -> float:
        return self.clock() - self.t0

    def resident_bytes(self) -> int:
        return sum(b for _, b in self.trees.values())

    def used(self) -> int:
        return self.in_use + self.resident_bytes() + sum(self.ws)

    def _note_peak(self):
        self.peak = max(self.peak, self.used())
        measure = getattr(self.ex, "measured_bytes", None)
        if measure is not None:
            m = measure()
            if m is not None:
                self.peak_measured = m if self.peak_measured is None else max(self.peak_measured, m)

    def submit(self, req: Request):
        if req.kind == "fit":
            req.footprint = self.ex.fit_footprint(req)
        else:
            req.footprint = self.ex.eval_footprint(req)
        self.pending.append(req)

    def _evict_for(self, need: int, protect: set) -> bool:
        """Drop least-recently-used trees until `need` fits.  Trees in
        `protect` and trees that a running evaluation reads stay."""
        protect = set(protect) | {r.tree for r, _ in self.running_evals}
        protect |= {r.tree for r in self.pending if r.kind == "eval"}
        while self.used() + need > self.budget:
            victim = next((rid for rid in self.trees if rid not in protect), None)
            if victim is None:
                return False
            tree, _ = self.trees.pop(victim)
            self.ex.release_tree(tree)
            self.evicted.add(victim)
        return True

    def _reject(self, req: Request, why: str):
        req.error = why
        req.done = self.now()
        self.finished.append(req)

    # --- one scheduling tick -------------------------------------------------
    def tick(self):
        now = self.now()
        # completions
        still = []
        for req, h in self.running_evals:
            if self.ex.done(h):
                req.result = self.ex.result(h)
                req.done = self.now()
                self.in_use -= req.footprint
                self.finished.append(req)
            else:
                still.append((req, h))
        self.running_evals = still
        running = []
        for reqs, h, slot in self.running_fits:
            if not self.ex.done(h):
                running.append((reqs, h, slot))
                continue
            trees = self.ex.result(h)
            t = self.now()
            for req, tree in zip(reqs, trees):
                self.in_use -= req.footprint
                if isinstance(tree, Exception):
                    req.error = str(tree)
                else:
                    # the fit's footprint counted its tree, so the tree fits
                    # once the footprint is released; if eviction still
                    # cannot make room, the tree is dropped, not kept over
                    # the budget
                    tb = self.ex.tree_bytes(req, tree)
                    if self._evict_for(tb, set()):
                        self.trees[req.rid] = (tree, tb)
                        req.result = tree
                        self._note_peak()
                    else:
                        self.ex.release_tree(tree)
                        req.error = "no device memory left for the fitted tree"
                req.done = t
                self.finished.append(req)
        self.running_fits = running
        # admission in arrival order; a request that cannot be admitted now
        # is skipped (later requests of the other kind may still go)
        fits: List[Request] = []
        fit_bytes = 0
        kept = collections.deque()
        busy = {slot for _, _, slot in self.running_fits}
        free_slots = [q for q in range(self.fit_slots) if q not in busy]
        blocked_fit = not free_slots
        slot = free_slots[0] if free_slots else -1
        ws_extra = 0   # growth of that stream's workspace for the batch being formed
        while self.pending:
            req = self.pending.popleft()
            if req.arrival > now:
                kept.append(req)
                continue
            if req.footprint > self.budget:
                self._reject(req, "request larger than the memory budget")
                continue
            if req.kind == "eval":
                if req.tree not in self.trees:
                    if req.tree in self.evicted or any(r.rid == req.tree for r in self.finished if r.error):
                        self._reject(req, "tree unavailable")
                    else:
                        kept.append(req)       # its fit has not finished yet
                    continue
                if len(self.running_evals) >= self.eval_slots:
                    kept.append(req)
                    self.deferred += 1
                    continue
                if not self._evict_for(req.footprint, {req.tree}):
                    kept.append(req)
                    self.deferred += 1
                    continue
                tree, tb = self.trees.pop(req.tree)
                self.trees[req.tree] = (tree, tb)          # most recently used
                req.admitted = self.now()
                self.in_use += req.footprint
                self._note_peak()
                self.running_evals.append((req, self.ex.start_eval(req, tree)))
            else:
                grow = 0
                if not blocked_fit:
                    need_ws = self.ex.workspace_bytes(fits + [req]) if hasattr(self.ex, "workspace_bytes") else 0
                    grow = max(0, need_ws - self.ws[slot])
                if blocked_fit or not self._evict_for(fit_bytes + req.footprint + grow, set()):
                    kept.append(req)
                    self.deferred += 1
                    continue
                fits.append(req)
                fit_bytes += req.footprint
                ws_extra = grow
        self.pending = kept
        if fits:
            for req in fits:
                req.admitted = self.now()
            self.in_use += fit_bytes
            self.ws[slot] += ws_extra
            self._note_peak()
            self.running_fits.append((fits, self.ex.start_fit_batch(fits, slot), slot))

    def idle(self) -> bool:
        return not self.pending and not self.running_evals and not self.running_fits

    def run(self, requests: List[Request], poll: float = 2e-4, timeout: float = 600.0):
        for r in sorted(requests, key=lambda r: r.arrival):
            self.submit(r)
        start = self.clock()
        while not self.idle():
            self.tick()
            if self.clock() - start > timeout:
                raise TimeoutError("serving loop did not drain")
            if poll:
                time.sleep(poll)
        return self.finished

    def stats(self) -> dict:
        out = {"peak_bytes": self.peak, "peak_measured_bytes": self.peak_measured, "budget_bytes": self.budget,
               "deferred": self.deferred}
        for kind in ("fit", "eval"):
            rs = [r for r in self.finished if r.kind == kind and r.error is None]
            lat = [r.latency for r in rs]
            if rs:
                span = max(r.done for r in rs) - min(r.arrival for r in rs)
                out[kind] = {"count": len(rs), "p50_ms": 1e3 * percentile(lat, 50),
                             "p99_ms": 1e3 * percentile(lat, 99),
                             "points_per_s": sum(r.n for r in rs) / span if span > 0 else float("nan")}
        return out


# ----------------------------------------------------------------------------
# the device executor
# ----------------------------------------------------------------------------
class GpuExecutor:
    """Runs admitted work through the library: batched fits on worker threads,
    one stream per fit slot, evaluations on a pool of streams (asynchronous).
    Device memory in use is measured as the device's used bytes less those
    in use when the executor was made."""

    def __init__(self, n_eval_streams: int = 4, device: str = "cuda:0", sort_queries: int = -1,
                 n_fit_streams: int = 2):
        import torch
        from . import fmt as F
        self.F = F
        self.torch = torch
        self.device = device
        F.load_library()
        self.fit_streams = [torch.cuda.Stream(device=device) for _ in range(n_fit_streams)]
        self.eval_streams = [torch.cuda.Stream(device=device) for _ in range(n_eval_streams)]
        self.next_stream = 0
        self.sort_queries = sort_queries
        torch.cuda.synchronize(device)
        free, total = torch.cuda.mem_get_info(device)
        self.base_used = total - free

    def measured_bytes(self) -> int:
        free, total = self.torch.cuda.mem_get_info(self.device)
        return int(total - free - self.base_used)

    # footprints
    def fit_footprint(self, req: Request) -> int:
        return fit_footprint(req.n, req.opts.get("p", 4), 4)

    def eval_footprint(self, req: Request) -> int:
        return eval_footprint(req.n, 4)

    def workspace_bytes(self, reqs: List[Request]) -> int:
        return workspace_footprint(sum(r.n for r in reqs), max(r.opts.get("p", 4) for r in reqs), 4)

    def tree_bytes(self, req: Request, tree) -> int:
        return tree_footprint(req.n, req.opts.get("p", 4))

    def release_tree(self, tree):
        tree.close()

    # fits: inputs (host numpy arrays) are copied on the fit stream by the worker
    def start_fit_batch(self, reqs: List[Request], slot: int = 0):
        torch, F = self.torch, self.F
        box = {"done": False, "trees": None}
        stream = self.fit_streams[slot % len(self.fit_streams)]

        def work():
            try:
                with torch.cuda.stream(stream):
                    xs, ys, zs, fs, opts = [], [], [], [], []
                    for r in reqs:
                        x, y, z, f = r.payload
                        xs.append(torch.from_numpy(x).to(self.device, non_blocking=False))
                        ys.append(torch.from_numpy(y).to(self.device, non_blocking=False))
                        zs.append(torch.from_numpy(z).to(self.device, non_blocking=False))
                        fs.append(torch.from_numpy(f).to(self.device, non_blocking=False))
                        opts.append(F.fmt_default_opts(**r.opts))
                    trees = F.fmt_fit_batch(opts, xs, ys, zs, fs, stream=stream)
                box["trees"] = trees
            except Exception as e:   # surfaced per request
                box["trees"] = [e] * len(reqs)
            box["done"] = True

        th = threading.Thread(target=work, daemon=True)
        th.start()
        return ("fit", box, th)

    def start_eval(self, req: Request, tree):
        torch, F = self.torch, self.F
        s = self.eval_streams[self.next_stream % len(self.eval_streams)]
        self.next_stream += 1
        qx, qy, qz = req.payload
        with torch.cuda.stream(s):
            dx = torch.from_numpy(qx).to(self.device, non_blocking=False)
            dy = torch.from_numpy(qy).to(self.device, non_blocking=False)
            dz = torch.from_numpy(qz).to(self.device, non_blocking=False)
            out = torch.empty(req.n, dtype=torch.float64, device=self.device)
            F.fmt_eval(tree, dx, dy, dz, out, self.sort_queries, stream=s)
            ev = torch.cuda.Event()
            ev.record(s)
        return ("eval", ev, (dx, dy, dz, out))

    def done(self, h) -> bool:
        if h[0] == "fit":
            return h[1]["done"]
        return h[1].query()

    def result(self, h):
        if h[0] == "fit":
            h[2].join()
            return h[1]["trees"]
        return h[2][3].cpu().numpy()


# ----------------------------------------------------------------------------
# request streams shaped like the served workload and a driver
# ----------------------------------------------------------------------------
def make_requests(seed: int, count: int, qps: float, fit_frac: float = 0.3, n_lo: float = 1e3,
                  n_hi: float = 1e6, nq_lo: float = 1e4, nq_hi: float = 1e6, p: int = 5,
                  warm_trees: int = 16, depth: int = 8, tol: float = 1e-8) -> List[Request]:
    """Poisson arrivals at `qps`; `warm_trees` fits arrive first (at t = 0),
    then fits (fraction `fit_frac`) and evaluations against any tree fitted
    so far.  Fit points come from seeded Gaussian mixtures with values from a
    seeded sum of Gaussian bumps; queries from the same mixture."""
    import math

    import synthetic
    rng = np.random.default_rng(seed)
    reqs: List[Request] = []
    rid = 0
    mixtures = {}

    def fit_req(t):
        nonlocal rid
        n = int(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi))))
        s = int(rng.integers(1 << 30))
        ncomp = int(rng.integers(1, 9))
        x, y, z = synthetic.mixture_points(n, s, ncomp, dtype=np.float32)
        b = synthetic.draw_bumps(s + 1)
        f = synthetic.bumps_value(b, x, y, z).astype(np.float32)
        mixtures[rid] = (s, ncomp)
        r = Request(rid=rid, kind="fit", arrival=t, n=n, payload=(x, y, z, f),
                    opts=dict(p=p, tol=tol, max_depth=depth))
        rid += 1
        return r

    for _ in range(warm_trees):
        reqs.append(fit_req(0.0))
    t = 0.0
    while len(reqs) < count:
        t += rng.exponential(1.0 / qps)
        if rng.uniform() < fit_frac:
            reqs.append(fit_req(t))
        else:
            fits = [r for r in reqs if r.kind == "fit"]
            target = fits[int(rng.integers(len(fits)))]
            nq = int(math.exp(rng.uniform(math.log(nq_lo), math.log(nq_hi))))
            s, ncomp = mixtures[target.rid]
            q = synthetic.mixture_points(nq, s + 7, ncomp, dtype=np.float32)
            reqs.append(Request(rid=rid, kind="eval", arrival=t, n=nq, payload=q, tree=target.rid))
            rid += 1
    return reqs


def serve_report(requests: int = 120, budget_gb: float = 16.0, streams: int = 4, seed: int = 4000,
                 loads=(0.5, 0.8), fit_slots: int = 2, progress=None) -> dict:
    """The served workload: a saturation run (every request arriving at
    once) measures the sustainable request rate, then Poisson streams at the
    given fractions of it report p50 / p99 latency, points per second, and the
    device memory in use (scheduler estimate and measured) against the
    budget."""
    ex = GpuExecutor(n_eval_streams=streams, n_fit_streams=fit_slots)
    budget = int(budget_gb * (1 << 30))
    reqs = make_requests(seed, requests, qps=1e9)
    srv = Server(ex, budget, eval_slots=streams, fit_slots=fit_slots)
    t0 = time.perf_counter()
    srv.run(reqs, poll=1e-4)
    span = time.perf_counter() - t0
    sat_qps = len(reqs) / span
    report = {"workload": "served stream: 30% fit (N log-uniform 1e3..1e6, mixtures, p=5), 70% eval "
                          "(1e4..1e6 queries), 16 warm trees, Poisson arrivals",
              "requests": requests, "fit_slots": fit_slots,
              "budget_bytes": budget, "eval_streams": streams,
              "saturation": {"requests_per_s": sat_qps, **srv.stats()}}
    for frac in loads:
        reqs = make_requests(seed + 1, requests, qps=frac * sat_qps)
        srv = Server(ex, budget, eval_slots=streams, fit_slots=fit_slots)
        srv.run(reqs, poll=1e-4)
        report[f"load_{frac:g}"] = {"qps": frac * sat_qps, **srv.stats()}
        if progress:
            progress(f"load {frac:g}: done")
    return report


def main():
    import argparse
    import json
    ap = argparse.ArgumentParser(description="serve a Poisson stream of fit/eval requests on one GPU")
    ap.add_argument("--requests", type=int, default=120)
    ap.add_argument("--budget-gb", type=float, default=16.0)
    ap.add_argument("--streams", type=int, default=4)
    ap.add_argument("--fit-slots", type=int, default=2)
    ap.add_argument("--seed", type=int, default=4000)
    ap.add_argument("--loads", type=str, default="0.5,0.8", help="fractions of the measured saturation rate")
    args = ap.parse_args()
    loads = [float(v) for v in args.loads.split(",") if v]
    report = serve_report(args.requests, args.budget_gb, args.streams, args.seed, loads, args.fit_slots,
                          progress=lambda m: print(m, flush=True))
    print(json.dumps(report))


if __name__ == "__main__":
    main()
