"""Write the oracle's expected values for the large clustered workload.

The workload: 2^26 points from a seeded 32-component Gaussian mixture (float32
storage), values from four anisotropic Gaussian bumps, p = 8, depth <= 10,
tol = 1e-8 (``synthetic.config5``).  This script calls only the CPU oracle
(``oracle.fit`` / ``oracle.evaluate``, Alg. 1 with Alg. 2 at every node) and
numpy; nothing here comes from the GPU library.  It stores, in
``config5_oracle.npz`` next to this file:

  * the oracle's node set (level, prefix, begin, count per node) and its
    rank flags;
  * the final residual at a seeded sample of the input points;
  * a seeded sample of the workload's 2^26 query points (their indices and
    coordinates), the oracle's evaluation there, and per sampled query the
    oracle-side statistics of its root-to-leaf chain: the largest leverage
    h = ||R^-T Lambda(u_q)||^2 (R: the triangle of Alg. 2's QR of the node's
    Vandermonde matrix, formed here by a streamed QR over row blocks), the
    largest condition number of the column-equilibrated triangle, and
    whether a node of the chain is rank-deficient;
  * the oracle's fit wall time and thread count.

Run (CPU only, about an hour on 8 cores):  python tests/golden/make_config5_golden.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synthetic  # noqa: E402
from oracle import fmt_oracle as fo  # noqa: E402

N_QUERY_SAMPLE = 1 << 15
N_POINT_SAMPLE = 1 << 15
BLOCK = 32768


def node_triangle(x, y, z, idx, c, s, p):
    """R of the QR of the node's Vandermonde matrix and its column norms, by
    QR of row blocks and of the stacked triangles."""
    tri = []
    cn2 = 0.0
    for b0 in range(0, idx.shape[0], BLOCK):
        sub = idx[b0:b0 + BLOCK]
        lam = oracle.moments((x[sub] - c[0]) * s[0], (y[sub] - c[1]) * s[1], (z[sub] - c[2]) * s[2], p)
        cn2 = cn2 + np.einsum("ij,ij->j", lam, lam)
        tri.append(np.linalg.qr(lam, mode="r"))
        if len(tri) >= 64:
            tri = [np.linalg.qr(np.vstack(tri), mode="r")]
    R = tri[0] if len(tri) == 1 else np.linalg.qr(np.vstack(tri), mode="r")
    return R, np.sqrt(cn2)


def main():
    t_start = time.time()
    pr = synthetic.config5(nq=0)
    x, y, z = (a.astype(np.float64) for a in (pr.x, pr.y, pr.z))
    print(f"inputs: n={pr.n} ({time.time() - t_start:.0f} s)", flush=True)
    t0 = time.time()
    ot = oracle.fit(pr.x, pr.y, pr.z, pr.f, pr.p, pr.tol, pr.max_depth)
    fit_s = time.time() - t0
    print(f"oracle fit: {ot.nodes} nodes, {int(ot.rank_deficient.sum())} rank-deficient, {fit_s:.0f} s", flush=True)

    # queries: the workload's 2^26 query points, drawn as synthetic.config5 draws them
    qx, qy, qz = synthetic.mixture_points(1 << 26, 5000 + 700, 32, dtype=np.float32)
    qsel = np.sort(np.random.default_rng(5005).choice(qx.shape[0], N_QUERY_SAMPLE, replace=False))
    sx, sy, sz = qx[qsel], qy[qsel], qz[qsel]
    del qx, qy, qz
    t0 = time.time()
    want = oracle.evaluate(ot, sx, sy, sz)
    print(f"oracle eval of {N_QUERY_SAMPLE} queries: {time.time() - t0:.0f} s", flush=True)

    # chain statistics of the sampled queries (oracle side only)
    D = ot.max_depth
    keys = oracle.morton(oracle.quantise(sx, 0.0, 1.0, D), oracle.quantise(sy, 0.0, 1.0, D),
                         oracle.quantise(sz, 0.0, 1.0, D), D)
    q = [a.astype(np.float64) for a in (sx, sy, sz)]
    h = np.zeros(N_QUERY_SAMPLE)
    kap = np.zeros(N_QUERY_SAMPLE)
    rank = np.zeros(N_QUERY_SAMPLE, dtype=bool)
    t0 = time.time()
    for i in range(ot.nodes):
        d, pre = int(ot.level[i]), int(ot.prefix[i])
        sel = (keys >> (3 * (D - d))) == pre
        if not np.any(sel):
            continue
        c, s = oracle.node_frame(d, fo._prefix_cell(pre, d), ot.lo, ot.hi)
        idx = ot.order[ot.begin[i]:ot.begin[i] + ot.count[i]]
        R, cn = node_triangle(x, y, z, idx, c, s, ot.p)
        sv = np.linalg.svd(R / cn[None, :], compute_uv=False)
        kap[sel] = np.maximum(kap[sel], sv[0] / max(sv[-1], 1e-300))
        if ot.rank_deficient[i]:
            rank[sel] = True
            continue
        lq = oracle.moments((q[0][sel] - c[0]) * s[0], (q[1][sel] - c[1]) * s[1], (q[2][sel] - c[2]) * s[2], ot.p)
        w = np.linalg.solve(R.T, lq.T)
        h[sel] = np.maximum(h[sel], np.sum(w * w, axis=0))
    print(f"chain statistics: {time.time() - t0:.0f} s", flush=True)

    psel = np.sort(np.random.default_rng(5006).choice(pr.n, N_POINT_SAMPLE, replace=False))
    try:
        from threadpoolctl import threadpool_info
        threads = max([dd.get("num_threads", 1) for dd in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    np.savez_compressed(
        os.path.join(HERE, "config5_oracle.npz"),
        level=ot.level.astype(np.uint8), prefix=ot.prefix.astype(np.uint32), begin=ot.begin.astype(np.uint32),
        count=ot.count.astype(np.uint32), rank_deficient=ot.rank_deficient,
        point_index=psel.astype(np.int64), residual=ot.residual[psel],
        query_index=qsel.astype(np.int64), qx=sx, qy=sy, qz=sz, want=want, h=h, kappa=kap, rank=rank,
        fit_seconds=np.float64(fit_s), threads=np.int64(threads))
    print(f"wrote config5_oracle.npz ({time.time() - t_start:.0f} s in all)", flush=True)


if __name__ == "__main__":
    main()
