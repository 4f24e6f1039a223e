"""The Gaussian-RBF factorisation (Section 2, eq. fullyfactored) on the GPU
through the C ABI: against the oracle's Lambda E T E Lambda^T element by
element (orders 0 to 14, ragged sizes, float32 and float64 points), and the
check it stands for: the truncated factorisation converges to the directly
evaluated Gaussian exp(-eps^2 |x_q - x_i|^2)."""
import numpy as np
import pytest

import oracle

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


def points(n, seed, dtype):
    rng = np.random.default_rng(seed)
    return [a.astype(dtype) for a in rng.uniform(-1.0, 1.0, (3, n))]


@pytest.mark.parametrize("p,eps,n,nq,dtype", [
    (0, 0.5, 130, 70, np.float64),
    (4, 0.5, 1000, 700, np.float64),      # ragged: neither size a multiple of the 64-tile
    (6, 0.3, 777, 129, np.float32),
    (8, 0.15, 1000, 700, np.float64),
    (10, 0.15, 300, 65, np.float64),
    (14, 0.15, 1000, 257, np.float64),    # calL = 680: eleven rounds of 64 basis entries
])
def test_rbf_factored_matches_oracle(fmt, p, eps, n, nq, dtype):
    print(f"[case] rbf p={p} eps={eps} n={n} nq={nq} {np.dtype(dtype).name}", flush=True)
    x = points(n, 100 + p, dtype)
    q = points(nq, 200 + p, dtype)
    got = fmt.fmt_rbf_factored(p, eps, *[dev(a) for a in x], *[dev(a) for a in q]).cpu().numpy()
    want = oracle.rbf_factored(*x, *q, p, eps)
    err = np.max(np.abs(got - want))
    print(f"max |gpu - oracle| {err:.3e} (max |phi'| {np.max(np.abs(want)):.3f})", flush=True)
    assert got.shape == (nq, n)
    assert err <= 1e-13 * max(1.0, float(np.max(np.abs(want))))


def test_rbf_factored_converges_to_the_gaussian(fmt):
    x = points(2000, 11, np.float64)
    q = points(500, 12, np.float64)
    d2 = sum((qa[:, None] - xa[None, :]) ** 2 for qa, xa in zip(q, x))
    eps = 0.15
    direct = np.exp(-eps * eps * d2)
    errs = []
    for p in (2, 6, 10, 14):
        got = fmt.fmt_rbf_factored(p, eps, *[dev(a) for a in x], *[dev(a) for a in q]).cpu().numpy()
        errs.append(float(np.max(np.abs(got - direct))))
    print(f"max |factored - Gaussian| by order 2, 6, 10, 14: {errs}", flush=True)
    assert errs[0] > errs[1] > errs[2] > errs[3]
    assert errs[3] < 1e-12


def test_rbf_factored_edges_and_errors(fmt):
    import torch
    x = [dev(a) for a in points(64, 1, np.float64)]
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    out = fmt.fmt_rbf_factored(4, 0.5, *x, e, e, e)      # no queries: nothing to do
    assert out.numel() == 0
    one = fmt.fmt_rbf_factored(0, 0.7, *x, *[t[:1] for t in x]).cpu().numpy()
    np.testing.assert_array_equal(one, np.ones((1, 64)))   # order 0: T = [1]
    for kw in (dict(p=15, eps=0.1), dict(p=4, eps=-1.0), dict(p=4, eps=float("inf"))):
        with pytest.raises(fmt.FmtError) as ex:
            fmt.fmt_rbf_factored(kw["p"], kw["eps"], *x, *x)
        assert ex.value.status == fmt.FMT_E_INVALID_ARG
