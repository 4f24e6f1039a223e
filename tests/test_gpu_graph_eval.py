"""fmt_eval_noalloc recorded into a HIP graph (torch.cuda.CUDAGraph) and
replayed: each replay, with eager work and synchronisations between the
replays and new query values written in place, equals the eager fmt_eval of
the same queries (bitwise), in input order and in sorted mode."""
import numpy as np
import pytest

import synthetic

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


@pytest.mark.parametrize("sort", [0, 1])
def test_eval_noalloc_graph_replays(fmt, sort):
    import torch
    pr = synthetic.small_problem(100000, 5, 91, tol=1e-8, depth=5, dtype=np.float32)
    print(f"[case] graph eval sort={sort}", flush=True)
    o = fmt.fmt_default_opts(p=pr.p, tol=pr.tol, max_depth=pr.max_depth)
    tree = fmt.fmt_fit(o, dev(pr.x), dev(pr.y), dev(pr.z), dev(pr.f))
    nq = 1 << 17
    Q = [dev(a) for a in synthetic.uniform_points(nq, 92, np.float32)]
    out = torch.empty(nq, dtype=torch.float64, device="cuda")
    fmt.fmt_eval(tree, *Q, out, sort_queries=sort)      # builds the evaluation tables
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        fmt.fmt_eval_noalloc(tree, *Q, out, sort_queries=sort, stream=s)   # warm-up outside the graph
        s.synchronize()
        with torch.cuda.graph(g, stream=s, capture_error_mode="relaxed"):
            fmt.fmt_eval_noalloc(tree, *Q, out, sort_queries=sort, stream=s)
    for rep in range(3):
        pts = synthetic.uniform_points(nq, 93 + rep, np.float32)
        for t, a in zip(Q, pts):
            t.copy_(torch.from_numpy(a))
        junk = torch.randn(1 << 20, device="cuda").sum()   # eager work between replays
        torch.cuda.synchronize()
        out.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        want = fmt.fmt_eval(tree, *Q, torch.empty(nq, dtype=torch.float64, device="cuda"),
                            sort_queries=sort).cpu().numpy()
        print(f"replay {rep}: equal {np.array_equal(got, want)} ({float(junk):.1f})", flush=True)
        np.testing.assert_array_equal(got, want)
    tree.close()
