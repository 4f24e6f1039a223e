"""Continuous batching on the GPU: requests served with overlap give the
same results as each request run alone (bitwise: a batched fit reduces
every problem's nodes in the same chunk order as a single fit, and
evaluation is deterministic); the device memory measured while serving stays
under the budget; a sample of the served fits matches the oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fmt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1511_01353_amd as m
    m.load_library()
    return m


def test_served_results_equal_alone(fmt):
    import torch

    from paper_1511_01353_amd.serve import GpuExecutor, Server, make_requests
    reqs = make_requests(seed=4242, count=20, qps=400.0, n_lo=2e3, n_hi=3e4, nq_lo=1e3, nq_hi=2e4,
                         warm_trees=4, depth=6)
    print(f"[case] serve {len(reqs)} requests", flush=True)
    ex = GpuExecutor(n_eval_streams=3)
    srv = Server(ex, budget_bytes=4 << 30, eval_slots=3)
    done = srv.run(reqs, poll=1e-4)
    assert len(done) == len(reqs)
    assert all(r.error is None for r in done), [r.error for r in done if r.error]
    assert srv.peak <= srv.budget
    # measured device memory (the device's used bytes less those in use
    # before serving), sampled at every admission, against the budget
    assert srv.peak_measured is not None and srv.peak_measured <= srv.budget
    st = srv.stats()
    print(st, flush=True)
    by = {r.rid: r for r in done}
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    alone = {}
    for r in reqs:
        if r.kind != "fit":
            continue
        x, y, z, f = r.payload
        t = fmt.fmt_fit(fmt.fmt_default_opts(**r.opts), dev(x), dev(y), dev(z), dev(f))
        alone[r.rid] = t
        served = by[r.rid].result
        a, b = served.export_points(), t.export_points()
        np.testing.assert_array_equal(a["residual"], b["residual"])
        np.testing.assert_array_equal(served.export_nodes()["coeffs"], t.export_nodes()["coeffs"])
    # the two smallest served fits against the oracle
    import oracle
    from test_gpu_parity import FP64_RMS, compare_topology
    fits = sorted([r for r in reqs if r.kind == "fit"], key=lambda r: r.n)[:2]
    for r in fits:
        x, y, z, f = r.payload
        print(f"[case] served fit {r.rid} against the oracle: n={r.n}", flush=True)
        ot = oracle.fit(x, y, z, f, r.opts["p"], r.opts["tol"], r.opts["max_depth"])
        _, pts = compare_topology(by[r.rid].result, ot)
        assert oracle.rms(pts["residual"] - ot.residual) <= FP64_RMS
    for r in reqs:
        if r.kind != "eval":
            continue
        qx, qy, qz = r.payload
        got = alone[r.tree].eval(dev(qx), dev(qy), dev(qz), sort_queries=-1).cpu().numpy()
        np.testing.assert_array_equal(by[r.rid].result, got)
