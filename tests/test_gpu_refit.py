"""Fixed-topology refit (fmt_refit) through the C ABI: new value fields on the
points of a fitted tree, its node set kept (the operator I' of Section 2,
eq. identityprime, through the tree's nodes), against the oracle's fit_fixed.

Bars as for the fit: topology and per-point outputs bit-exact (they are the
tree's), float64 fitted values and evaluations within RMS 1e-10 of the
oracle; the fields of one call equal single-field calls bit for bit.
"""
import numpy as np
import pytest

import oracle
import synthetic
from test_gpu_parity import FP64_RMS, compare_eval, compare_topology, dev, oracle_fit, print_case, run_fit
from test_oracle_pins import poly_derivative_at, poly_eval, random_poly

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fmt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1511_01353_amd as m
    m.load_library()
    return m


def new_fields(pr, seeds):
    """Fields other than the one the tree was built from: Gaussian bumps of
    other seeds and the Franke function, in the problem's dtype."""
    out = []
    for s in seeds:
        if s < 0:
            v = synthetic.franke3d(pr.x, pr.y, pr.z)
        else:
            v = synthetic.bumps_value(synthetic.draw_bumps(s), pr.x, pr.y, pr.z)
        out.append(np.asarray(v, dtype=pr.x.dtype))
    return np.stack(out)


def refit(fmt, tr, pr, fields):
    return fmt.fmt_refit(tr, dev(pr.x), dev(pr.y), dev(pr.z), dev(np.ascontiguousarray(fields)))


def same_topology(a, b):
    na, nb = a.export_nodes(), b.export_nodes()
    for k in ("level", "prefix", "begin", "count"):
        np.testing.assert_array_equal(na[k], nb[k])
    pa, pb = a.export_points(), b.export_points()
    for k in ("keys", "order", "leaf"):
        np.testing.assert_array_equal(pa[k], pb[k])
    return na, pa


@pytest.mark.parametrize("n,p,depth,tol,seed,dtype,clustered", [
    (20000, 4, 4, 1e-7, 11, np.float32, False),
    (30000, 6, 4, 1e-8, 12, np.float64, False),
    (6000, 2, 3, 1e-9, 13, np.float32, False),
    (30000, 4, 5, 1e-7, 31, np.float32, True),     # clustered: deflated nodes on faces
])
def test_refit_matches_oracle(fmt, n, p, depth, tol, seed, dtype, clustered):
    pr = synthetic.small_problem(n, p, seed, tol=tol, depth=depth, dtype=dtype, clustered=clustered, nq=4000)
    print_case("refit", pr)
    tr = run_fit(fmt, pr)
    ot = oracle_fit(pr)
    compare_topology(tr, ot)
    fields = new_fields(pr, [seed + 100, -1])
    outs = refit(fmt, tr, pr, fields)
    assert len(outs) == 2
    for out, f in zip(outs, fields):
        nodes, pts = same_topology(out, tr)
        ow = oracle.fit_fixed(ot, pr.x, pr.y, pr.z, f)
        f64 = f.astype(np.float64)
        err = oracle.rms((f64 - pts["residual"]) - (f64 - ow.residual))
        print(f"fitted values rms diff {err:.3e}", flush=True)
        assert err <= FP64_RMS
        got = out.eval(dev(pr.qx), dev(pr.qy), dev(pr.qz)).cpu().numpy()
        compare_eval(ow, nodes, pr, got, oracle.evaluate(ow, pr.qx, pr.qy, pr.qz), FP64_RMS, min_frac=0.85)
        out.close()
    tr.close()


def test_refit_of_own_values_reproduces_fit(fmt):
    pr = synthetic.small_problem(200000, 6, 21, tol=1e-8, depth=5, dtype=np.float32)
    print_case("refit-own", pr)
    tr = run_fit(fmt, pr)
    (out,) = refit(fmt, tr, pr, pr.f[None, :])
    na, _ = same_topology(out, tr)
    nb = tr.export_nodes()
    ok = (nb["flags"] & 1) == 0
    scale = np.maximum(np.abs(nb["coeffs"][ok]), 1.0)
    assert np.max(np.abs(na["coeffs"][ok] - nb["coeffs"][ok]) / scale) < 1e-7
    ra, rb = out.export_points()["residual"], tr.export_points()["residual"]
    assert oracle.rms(ra - rb) <= 1e-11


def test_refit_fields_independent_and_linear(fmt):
    pr = synthetic.small_problem(50000, 5, 23, tol=1e-8, depth=4, dtype=np.float64)
    print_case("refit-linear", pr)
    tr = run_fit(fmt, pr)
    a, b = new_fields(pr, [7, 8])
    outs = refit(fmt, tr, pr, np.stack([a, b, 2.0 * a - 3.0 * b]))
    (single,) = refit(fmt, tr, pr, b[None, :])
    ca, cb, cc = (o.export_nodes()["coeffs"] for o in outs)
    np.testing.assert_array_equal(cb, single.export_nodes()["coeffs"])
    np.testing.assert_array_equal(outs[1].export_points()["residual"], single.export_points()["residual"])
    scale = np.max(np.abs(2.0 * ca)) + np.max(np.abs(3.0 * cb))
    assert np.max(np.abs(cc - (2.0 * ca - 3.0 * cb))) < 1e-11 * scale


def test_refit_polynomial_field(fmt):
    """A degree <= p field on a split tree: the root takes the node-frame
    Taylor coefficients (closed form), every other node ~0."""
    pr = synthetic.small_problem(40000, 4, 25, tol=1e-8, depth=4, dtype=np.float64)
    tr = run_fit(fmt, pr)
    assert tr.info().nodes > 9
    poly = random_poly(pr.p, 9)
    (out,) = refit(fmt, tr, pr, poly_eval(poly, pr.x, pr.y, pr.z)[None, :])
    c = out.export_nodes()["coeffs"]
    for j, e in enumerate(oracle.exponents(pr.p)):
        want = poly_derivative_at(poly, e, (0.5, 0.5, 0.5)) * 0.5 ** sum(e)
        assert abs(c[0, j] - want) < 1e-10, (e, c[0, j], want)
    assert np.max(np.abs(c[1:])) < 1e-9
    assert oracle.max_abs(out.export_points()["residual"]) < 1e-11


def test_refit_batch_member_equals_single(fmt):
    probs = synthetic.config3(seed0=3100, count=4, nlo=2e3, nhi=3e4, nq=500)
    opts = [fmt.fmt_default_opts(p=pr.p, tol=pr.tol, max_depth=pr.max_depth) for pr in probs]
    trees = fmt.fmt_fit_batch(opts, [dev(p.x) for p in probs], [dev(p.y) for p in probs],
                              [dev(p.z) for p in probs], [dev(p.f) for p in probs])
    for k, (pr, tb) in enumerate(zip(probs, trees)):
        ts = run_fit(fmt, pr)
        fields = new_fields(pr, [400 + k])
        (ob,) = refit(fmt, tb, pr, fields)
        (os_,) = refit(fmt, ts, pr, fields)
        same_topology(ob, os_)
        np.testing.assert_array_equal(ob.export_nodes()["coeffs"], os_.export_nodes()["coeffs"])
        np.testing.assert_array_equal(ob.export_points()["residual"], os_.export_points()["residual"])


def test_refit_errors(fmt):
    pr = synthetic.small_problem(8000, 3, 27, tol=1e-7, depth=3, dtype=np.float64)
    tr = run_fit(fmt, pr)
    f = new_fields(pr, [1])
    with pytest.raises(fmt.FmtError) as e:   # a point moved to another cell
        x = pr.x.copy()
        x[5] = 1.0 - x[5]
        fmt.fmt_refit(tr, dev(x), dev(pr.y), dev(pr.z), dev(f))
    assert e.value.status == fmt.FMT_E_INVALID_ARG
    with pytest.raises(fmt.FmtError) as e:   # another point count
        fmt.fmt_refit(tr, dev(pr.x[:-1]), dev(pr.y[:-1]), dev(pr.z[:-1]), dev(f[:, :-1]))
    assert e.value.status == fmt.FMT_E_INVALID_ARG
    nodes = tr.export_nodes()
    ti = fmt.fmt_tree_import(fmt.fmt_default_opts(p=pr.p, max_depth=pr.max_depth), nodes["level"],
                             nodes["prefix"], nodes["coeffs"])
    with pytest.raises(fmt.FmtError) as e:   # an imported tree holds no points
        fmt.fmt_refit(ti, dev(pr.x), dev(pr.y), dev(pr.z), dev(f))
    assert e.value.status == fmt.FMT_E_INVALID_ARG
    fb = f.copy()
    fb[0, 123] = np.nan
    with pytest.raises(fmt.FmtError) as e:   # a non-finite value
        fmt.fmt_refit(tr, dev(pr.x), dev(pr.y), dev(pr.z), dev(fb))
    assert e.value.status == fmt.FMT_E_NUMERIC
    # the tree still refits after the failures
    (out,) = refit(fmt, tr, pr, f)
    same_topology(out, tr)


def test_refit_full_size_properties(fmt):
    """The benchmark's workload (2^20 points, p = 6, 3 414 nodes), where the
    oracle is too slow to refit: the refit of the fit's own values reproduces
    the fit, and a new field's final residual is orthogonal to the basis of
    sampled leaves (each leaf's residual is its own least-squares residual,
    so Lambda^T r = 0 up to rounding)."""
    pr = synthetic.config2(nq=1000)
    print_case("refit-full", pr)
    tr = run_fit(fmt, pr)
    f2 = new_fields(pr, [77])[0]
    own, new = refit(fmt, tr, pr, np.stack([pr.f, f2]))
    nb = tr.export_nodes()
    na, _ = same_topology(own, tr)
    ok = (nb["flags"] & 1) == 0
    scale = np.maximum(np.abs(nb["coeffs"][ok]), 1.0)
    assert np.max(np.abs(na["coeffs"][ok] - nb["coeffs"][ok]) / scale) < 1e-7
    assert oracle.rms(own.export_points()["residual"] - tr.export_points()["residual"]) <= 1e-11
    nn, pn = same_topology(new, tr)
    level = nn["level"].astype(np.int64)
    prefix = nn["prefix"].astype(np.int64)
    parents = {(int(l) - 1, int(q) >> 3) for l, q in zip(level, prefix) if l > 0}
    leaves = [i for i in range(len(level)) if (int(level[i]), int(prefix[i])) not in parents]
    rng = np.random.default_rng(5)
    from oracle import fmt_oracle as fo
    x, y, z = (np.asarray(a, np.float64) for a in (pr.x, pr.y, pr.z))
    r = pn["residual"]
    order = pn["order"].astype(np.int64)
    for i in rng.choice(leaves, 16, replace=False):
        idx = order[nn["begin"][i]:nn["begin"][i] + nn["count"][i]]
        c, s = oracle.node_frame(int(level[i]), fo._prefix_cell(int(prefix[i]), int(level[i])), (0, 0, 0), (1, 1, 1))
        lam = oracle.moments((x[idx] - c[0]) * s[0], (y[idx] - c[1]) * s[1], (z[idx] - c[2]) * s[2], pr.p)
        g = lam.T @ r[idx]
        bound = 1e-10 * np.linalg.norm(lam) * np.linalg.norm(f2[idx].astype(np.float64))
        assert np.max(np.abs(g)) <= bound, (i, np.max(np.abs(g)), bound)
