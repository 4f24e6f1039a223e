"""fmt_eval_noalloc (the evaluation entry point that allocates nothing)
against fmt_eval, through the C ABI: two calls in a row, the second with a
smaller input, in sorted mode (the mode that uses the scratch array) and in
input order, float32 and float64 queries; the error paths (tables not built
yet, a sorted request beyond the scratch array)."""
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


def test_eval_noalloc_equals_eval(fmt):
    import torch
    pr = synthetic.small_problem(200000, 6, 77, tol=1e-8, depth=5, dtype=np.float32)
    print(f"[case] no-alloc eval: n={pr.n} p={pr.p} D={pr.max_depth}", flush=True)
    o = fmt.fmt_default_opts(p=pr.p, tol=pr.tol, max_depth=pr.max_depth)
    tree = fmt.fmt_fit(o, dev(pr.x), dev(pr.y), dev(pr.z), dev(pr.f))
    q32 = synthetic.uniform_points(1 << 20, 78, np.float32)
    Q = [dev(a) for a in q32]
    out = torch.empty(1 << 20, dtype=torch.float64, device="cuda")
    # before the first fmt_eval the tree's evaluation tables do not exist
    with pytest.raises(fmt.FmtError) as e:
        fmt.fmt_eval_noalloc(tree, *Q, out, sort_queries=1)
    assert e.value.status == fmt.FMT_E_INVALID_ARG
    # two calls in a row, the second smaller (the array keeps the first's
    # contents), each against fmt_eval on the same queries
    cases = [(Q, 1 << 20, np.float32), (None, 1 << 17, np.float64)]
    for i, (qq, n, dt) in enumerate(cases):
        if qq is None:
            qq = [dev(a) for a in synthetic.uniform_points(n, 79 + i, dt)]
        for sort in (1, 0):
            want = fmt.fmt_eval(tree, qq[0], qq[1], qq[2],
                                torch.empty(n, dtype=torch.float64, device="cuda"), sort_queries=sort)
            got = fmt.fmt_eval_noalloc(tree, qq[0], qq[1], qq[2],
                                       torch.full((n,), np.nan, dtype=torch.float64, device="cuda"),
                                       sort_queries=sort)
            torch.cuda.synchronize()
            print(f"call {i}: n={n} {np.dtype(dt).name} sort={sort}", flush=True)
            np.testing.assert_array_equal(got.cpu().numpy(), want.cpu().numpy())
    # the largest sorted float64 request the array holds, then one beyond it
    qq = [dev(a) for a in synthetic.uniform_points(1 << 20, 81, np.float64)]
    want = fmt.fmt_eval(tree, *qq, torch.empty(1 << 20, dtype=torch.float64, device="cuda"), sort_queries=1)
    got = fmt.fmt_eval_noalloc(tree, *qq, torch.empty(1 << 20, dtype=torch.float64, device="cuda"), sort_queries=1)
    np.testing.assert_array_equal(got.cpu().numpy(), want.cpu().numpy())
    big = [dev(a) for a in synthetic.uniform_points(1 << 21, 82, np.float64)]
    with pytest.raises(fmt.FmtError) as e:
        fmt.fmt_eval_noalloc(tree, *big, torch.empty(1 << 21, dtype=torch.float64, device="cuda"), sort_queries=1)
    assert e.value.status == fmt.FMT_E_INVALID_ARG
    tree.close()
