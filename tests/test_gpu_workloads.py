"""Full-size runs of the batched and the large clustered workloads.

Batched (256 uneven problems in one batched fit): every problem is checked
against properties that hold at any size (keys, order and topology against
their integer definitions; evaluation at the data points equals f - r), and a
sample of problems against the oracle element by element.

Large clustered (2^26 points, p = 8, depth <= 10): the oracle needs 4.4 hours
of the host for it (tests/golden/make_config5_golden.py), so the test
compares with the oracle's stored results: its node set bit for bit, the
final residual at 2^15 sampled points, and the evaluation at 2^15 sampled
queries of the workload on the queries the data determine (the oracle-side
chain statistics stored with them decide which).  Besides, properties that
hold at any size: keys on a sample against their definition, the order sorts
the keys, every node's range and count against the sorted keys, points'
leaves, non-root nodes hold at least calL points, evaluation at sampled data
points equals f - r, sorted and unsorted evaluation agree bitwise, and at
sampled nodes the residual right after the node's fit is orthogonal to the
node's basis (the normal equations of Alg. 2's least-squares problem).
"""
import os
import time
from types import SimpleNamespace

import numpy as np
import pytest

import oracle
import synthetic
from test_gpu_parity import FP64_RMS, compare_eval, compare_topology, fitted_rms, oracle_fit

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fmt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1511_01353_amd as m
    m.load_library()
    return m


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def check_keys_and_topology(pr, tr, nodes, pts, sample=None, rng=None):
    """Integer work against its definition: keys (all points or a sample),
    the order sorts them, every node's begin/count is the range of sorted
    keys with its prefix, leaves are the deepest nodes holding the points,
    non-root nodes hold at least calL points."""
    D, p = pr.max_depth, pr.p
    L = oracle.basis_size(p)
    keys = pts["keys"].astype(np.int64)
    idx = np.arange(pr.n) if sample is None else rng.choice(pr.n, sample, replace=False)
    want = oracle.morton(oracle.quantise(pr.x[idx], 0.0, 1.0, D), oracle.quantise(pr.y[idx], 0.0, 1.0, D),
                         oracle.quantise(pr.z[idx], 0.0, 1.0, D), D)
    np.testing.assert_array_equal(keys[idx], want)
    order = pts["order"].astype(np.int64)
    assert np.array_equal(np.sort(order), np.arange(pr.n))
    sk = keys[order]
    assert np.all(np.diff(sk) >= 0)
    level = nodes["level"].astype(np.int64)
    prefix = nodes["prefix"].astype(np.int64)
    assert level[0] == 0 and nodes["begin"][0] == 0 and nodes["count"][0] == pr.n
    for d in range(1, int(level.max()) + 1):
        sel = np.nonzero(level == d)[0]
        top = sk >> (3 * (D - d))
        lo = np.searchsorted(top, prefix[sel], side="left")
        hi = np.searchsorted(top, prefix[sel], side="right")
        np.testing.assert_array_equal(nodes["begin"][sel].astype(np.int64), lo)
        np.testing.assert_array_equal(nodes["count"][sel].astype(np.int64), hi - lo)
        assert np.all(hi - lo >= L)
        # the parent exists
        par = prefix[sel] >> 3
        up = np.sort(prefix[level == d - 1])
        pos = np.searchsorted(up, par)
        assert np.all(up[np.minimum(pos, len(up) - 1)] == par)
    # leaves of the sampled points: the deepest node whose prefix holds the key
    leaf = np.zeros(idx.shape[0], np.int64)
    for d in range(0, int(level.max()) + 1):
        sel = np.nonzero(level == d)[0]
        order_d = np.argsort(prefix[sel])
        ps = prefix[sel][order_d]
        k = keys[idx] >> (3 * (D - d))
        pos = np.minimum(np.searchsorted(ps, k), len(ps) - 1)
        hit = ps[pos] == k
        leaf[hit] = sel[order_d][pos[hit]]
    np.testing.assert_array_equal(pts["leaf"][idx].astype(np.int64), leaf)


def check_eval_at_points(pr, tr, pts, rng, count):
    sel = rng.choice(pr.n, min(pr.n, count), replace=False)
    got = tr.eval(dev(pr.x[sel]), dev(pr.y[sel]), dev(pr.z[sel])).cpu().numpy()
    want = pr.f[sel].astype(np.float64) - pts["residual"][sel]
    err = np.max(np.abs(got - want))
    scale = max(1.0, float(np.max(np.abs(pr.f))))
    assert err <= 1e-9 * scale, err
    return err


def test_nearly_singular_node_keeps_its_accuracy(fmt):
    """Problem 70 of the batched workload (7 921 mixture points, p = 6) has a
    node of 134 points whose equilibrated normal equations carry pivots at the
    rounding level; a factorisation whose two triangles drift apart under
    rounding kept one of them there and lost three digits of the fit
    (coefficients of 2e9, residual RMS 0.11).  The GPU's deflation and the
    oracle's Householder QR treat that node differently (its condition is
    beyond either's rank threshold), so one child more activates on the GPU
    and the node sets differ; what the data determine is compared: the final
    residual's RMS against the oracle's, moderate coefficients, and
    evaluation at the data points equal to f - r."""
    pr = synthetic.config3()[70]
    print(f"[case] {pr.name}: n={pr.n} p={pr.p}", flush=True)
    o = fmt.fmt_default_opts(p=pr.p, tol=pr.tol, max_depth=pr.max_depth)
    tr = fmt.fmt_fit(o, dev(pr.x), dev(pr.y), dev(pr.z), dev(pr.f))
    ot = oracle.fit(pr.x, pr.y, pr.z, pr.f, pr.p, pr.tol, pr.max_depth)
    nodes, pts = tr.export_nodes(), tr.export_points()
    r_gpu, r_or = oracle.rms(pts["residual"]), oracle.rms(ot.residual)
    cmax = float(np.max(np.abs(nodes["coeffs"])))
    print(f"nodes {len(nodes['level'])} (oracle {ot.nodes}); residual rms {r_gpu:.4e} (oracle {r_or:.4e}); "
          f"max |coef| {cmax:.3e}", flush=True)
    assert r_gpu <= 1.05 * r_or
    assert cmax < 1e7
    check_eval_at_points(pr, tr, pts, np.random.default_rng(70), pr.n)
    tr.close()


def test_batched_workload(fmt):
    import torch
    probs = synthetic.config3()
    total = sum(pr.n for pr in probs)
    print(f"[case] batched: {len(probs)} problems, {total} points", flush=True)
    opts = [fmt.fmt_default_opts(p=pr.p, tol=pr.tol, max_depth=pr.max_depth) for pr in probs]
    X = [dev(pr.x) for pr in probs]
    Y = [dev(pr.y) for pr in probs]
    Z = [dev(pr.z) for pr in probs]
    Fv = [dev(pr.f) for pr in probs]
    fmt.fmt_fit_batch(opts, X, Y, Z, Fv)   # warm-up (workspace, code)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    trees = fmt.fmt_fit_batch(opts, X, Y, Z, Fv)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    nodes_total = sum(int(t.info().nodes) for t in trees)
    print(f"batched fit: {total / dt:.3e} points/s ({dt * 1e3:.1f} ms, {nodes_total} nodes)", flush=True)
    rng = np.random.default_rng(3)
    worst = 0.0
    for pr, tr in zip(probs, trees):
        nodes, pts = tr.export_nodes(), tr.export_points()
        check_keys_and_topology(pr, tr, nodes, pts)
        worst = max(worst, check_eval_at_points(pr, tr, pts, rng, 512))
    print(f"eval at data points vs f - r: max diff {worst:.2e}", flush=True)
    # oracle parity on a sample: the smallest and the median problem of each
    # degree.  The queries come from the problem's mixture, so in the smallest
    # problems many fall far outside their leaf's points (leverage above the
    # bound) or under a node whose points are coplanar on a clipped face (the
    # oracle's rank flag): measured coverage is 0.365 at least (problem 29:
    # 1 017 points, p = 6), hence the floor of 0.3.
    for p in (4, 5, 6):
        ks = sorted([k for k, pr in enumerate(probs) if pr.p == p], key=lambda k: probs[k].n)
        for k in (ks[0], ks[len(ks) // 2]):
            pr, tr = probs[k], trees[k]
            print(f"[case] batched problem {k}: n={pr.n} p={pr.p}", flush=True)
            ot = oracle_fit(pr)
            nodes, pts = compare_topology(tr, ot)
            assert fitted_rms(pr, pts, ot) <= FP64_RMS
            want = oracle.evaluate(ot, pr.qx, pr.qy, pr.qz)
            got = tr.eval(dev(pr.qx), dev(pr.qy), dev(pr.qz)).cpu().numpy()
            compare_eval(ot, nodes, pr, got, want, FP64_RMS, min_frac=0.3)
    # a problem's bits do not depend on its batch: at this size the levels
    # are laid out by the tiled topology launches and the late refinement
    # runs over listed nodes, neither of which a single fit of one of these
    # problems does
    for p in (4, 5, 6):
        ks = sorted([k for k, pr in enumerate(probs) if pr.p == p], key=lambda k: probs[k].n)
        for k in (ks[len(ks) // 2], ks[-1]):
            pr, tb = probs[k], trees[k]
            print(f"[case] batched problem {k} against its single fit: n={pr.n} p={pr.p}", flush=True)
            ts = fmt.fmt_fit(opts[k], X[k], Y[k], Z[k], Fv[k])
            a, b = tb.export_points(), ts.export_points()
            for key in ("keys", "leaf", "residual"):
                np.testing.assert_array_equal(a[key], b[key])
            np.testing.assert_array_equal(tb.export_nodes()["coeffs"], ts.export_nodes()["coeffs"])
            ts.close()
    for tr in trees:
        tr.close()


def lam(pr, x, y, z, level, prefix):
    """Basis values of a node's frame at points (the definition of Section 2)."""
    from oracle import fmt_oracle as fo
    c, s = oracle.node_frame(level, fo._prefix_cell(prefix, level), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0))
    return oracle.moments((x - c[0]) * s[0], (y - c[1]) * s[1], (z - c[2]) * s[2], pr.p)


def test_large_clustered_workload(fmt):
    import torch
    t0 = time.perf_counter()
    pr = synthetic.config5(nq=1 << 22)
    print(f"[case] large clustered: n={pr.n} p={pr.p} D={pr.max_depth} (inputs in {time.perf_counter() - t0:.0f} s)",
          flush=True)
    o = fmt.fmt_default_opts(p=pr.p, tol=pr.tol, max_depth=pr.max_depth)
    X, Y, Z, Fv = dev(pr.x), dev(pr.y), dev(pr.z), dev(pr.f)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tr = fmt.fmt_fit(o, X, Y, Z, Fv)
    dt = time.perf_counter() - t0
    info = tr.info()
    print(f"fit: {pr.n / dt:.3e} points/s ({dt * 1e3:.0f} ms), {info.nodes} nodes, per level "
          f"{[int(info.per_level[i]) for i in range(info.depth + 1)]}", flush=True)
    QX, QY, QZ = dev(pr.qx), dev(pr.qy), dev(pr.qz)
    out = torch.empty(QX.numel(), dtype=torch.float64, device="cuda")
    tr.eval(QX, QY, QZ, out=out)   # first evaluation builds the composite coefficients
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tr.eval(QX, QY, QZ, out=out, sort_queries=1)
    torch.cuda.synchronize()
    dq = time.perf_counter() - t0
    fq = out.cpu().numpy()
    assert np.all(np.isfinite(fq))
    print(f"eval (sorted): {QX.numel() / dq:.3e} queries/s; E_rms vs truth "
          f"{oracle.rms(fq - pr.qf_true):.3e}", flush=True)
    nq = 1 << 20
    a = tr.eval(QX[:nq], QY[:nq], QZ[:nq], sort_queries=1).cpu().numpy()
    b = tr.eval(QX[:nq], QY[:nq], QZ[:nq], sort_queries=0).cpu().numpy()
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(a, fq[:nq])

    nodes, pts = tr.export_nodes(), tr.export_points()
    rng = np.random.default_rng(5)
    check_keys_and_topology(pr, tr, nodes, pts, sample=1 << 20, rng=rng)
    err = check_eval_at_points(pr, tr, pts, rng, 1 << 20)
    print(f"eval at data points vs f - r: max diff {err:.2e}", flush=True)

    # normal equations at sampled nodes: Lambda^T r_after ~ 0, where r_after
    # (right after the node's fit) is the final residual plus the polynomials
    # of the node's descendants
    level = nodes["level"].astype(np.int64)
    prefix = nodes["prefix"].astype(np.int64)
    count = nodes["count"].astype(np.int64)
    D = pr.max_depth
    keys = pts["keys"].astype(np.int64)
    sk_order = pts["order"].astype(np.int64)
    x = pr.x.astype(np.float64)
    y = pr.y.astype(np.float64)
    z = pr.z.astype(np.float64)
    cand = np.nonzero((count <= 200000))[0]
    picks = rng.choice(cand, size=min(12, cand.shape[0]), replace=False)
    for i in picks:
        d, pre = int(level[i]), int(prefix[i])
        b0 = int(nodes["begin"][i])
        ids = sk_order[b0:b0 + int(count[i])]
        r_after = pts["residual"][ids].copy()
        desc = np.nonzero((level > d) & ((prefix >> (3 * np.maximum(level - d, 0))) == pre))[0]
        for j in desc:
            dj, pj = int(level[j]), int(prefix[j])
            inside = (keys[ids] >> (3 * (D - dj))) == pj
            if np.any(inside):
                sub = ids[inside]
                r_after[inside] += lam(pr, x[sub], y[sub], z[sub], dj, pj) @ nodes["coeffs"][j]
        A = lam(pr, x[ids], y[ids], z[ids], d, pre)
        r_before = r_after + A @ nodes["coeffs"][i]
        g_after = np.linalg.norm(A.T @ r_after)
        g_before = np.linalg.norm(A.T @ r_before)
        floor = 1e-12 * np.linalg.norm(A) * np.sqrt(ids.shape[0]) * max(1.0, float(np.max(np.abs(pr.f))))
        print(f"node level {d} n={ids.shape[0]} descendants={desc.shape[0]}: |A^T r_after| {g_after:.2e} "
              f"(|A^T r_before| {g_before:.2e}, floor {floor:.2e})", flush=True)
        assert g_after <= 1e-6 * g_before + floor
        assert np.linalg.norm(r_after) <= np.linalg.norm(r_before) * (1 + 1e-12)

    # against the oracle's stored results (written by a script that calls
    # only the oracle): node set, residual at sampled points, evaluation at
    # sampled queries
    golden = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "config5_oracle.npz")
    g = np.load(golden)
    print(f"stored oracle: {g['level'].shape[0]} nodes, fitted in {float(g['fit_seconds']):.0f} s on "
          f"{int(g['threads'])} threads", flush=True)
    assert level.shape[0] == g["level"].shape[0]
    np.testing.assert_array_equal(level, g["level"].astype(np.int64))
    np.testing.assert_array_equal(prefix, g["prefix"].astype(np.int64))
    np.testing.assert_array_equal(nodes["begin"].astype(np.int64), g["begin"].astype(np.int64))
    np.testing.assert_array_equal(count, g["count"].astype(np.int64))
    pi = g["point_index"]
    res_rms = oracle.rms(pts["residual"][pi] - g["residual"])
    print(f"residual at {pi.shape[0]} sampled points: rms diff {res_rms:.3e}", flush=True)
    assert res_rms <= FP64_RMS
    gq = tr.eval(dev(g["qx"]), dev(g["qy"]), dev(g["qz"])).cpu().numpy()
    keys_q = oracle.morton(oracle.quantise(g["qx"], 0.0, 1.0, D), oracle.quantise(g["qy"], 0.0, 1.0, D),
                           oracle.quantise(g["qz"], 0.0, 1.0, D), D)
    ot = SimpleNamespace(max_depth=D, level=g["level"].astype(np.int64), prefix=g["prefix"].astype(np.int64),
                         rank_deficient=g["rank_deficient"])
    compare_eval(ot, nodes, pr, gq, g["want"], FP64_RMS, min_frac=0.95,   # measured coverage 0.991
                 stats=(g["h"], g["kappa"], g["rank"], keys_q))
    tr.close()
