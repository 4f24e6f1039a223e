"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-types an oracle formula: each compares the oracle with a
printed value, a closed form, an exact rational computation, a different
library routine, or an invariant the method guarantees.  The mutation tests at
the bottom plant plausible mistakes in the oracle (on the CPU) and check that
at least one pin fails for each.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import fmt_oracle as fo
import synthetic

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------------------
# helpers that are independent of the oracle
# ----------------------------------------------------------------------------
def brute_monomials(p):
    """All (l, m, n) with l+m+n <= p by brute force (no ordering assumed)."""
    return {(l, m, n) for l in range(p + 1) for m in range(p + 1) for n in range(p + 1) if l + m + n <= p}


def random_poly(p, seed):
    """A random polynomial of total degree <= p as {(a,b,c): coef} in global x, y, z."""
    rng = np.random.default_rng(seed)
    return {e: float(rng.uniform(-1, 1)) for e in brute_monomials(p)}


def poly_eval(poly, x, y, z):
    out = np.zeros_like(np.asarray(x, dtype=np.float64))
    for (a, b, c), k in poly.items():
        out += k * x ** a * y ** b * z ** c
    return out


def poly_derivative_at(poly, alpha, pt):
    """d^alpha poly at pt (exact differentiation of each monomial)."""
    l, m, n = alpha
    tot = 0.0
    for (a, b, c), k in poly.items():
        if a < l or b < m or c < n:
            continue
        fa = math.factorial(a) // math.factorial(a - l)
        fb = math.factorial(b) // math.factorial(b - m)
        fc = math.factorial(c) // math.factorial(c - n)
        tot += k * fa * fb * fc * pt[0] ** (a - l) * pt[1] ** (b - m) * pt[2] ** (c - n)
    return tot


def exact_lstsq(rows, rhs):
    """Exact least squares over the rationals: solve (A^T A) x = A^T b by Gauss-Jordan."""
    n = len(rows[0])
    ata = [[sum(r[i] * r[j] for r in rows) for j in range(n)] for i in range(n)]
    atb = [sum(r[i] * b for r, b in zip(rows, rhs)) for i in range(n)]
    M = [ata[i] + [atb[i]] for i in range(n)]
    for c in range(n):
        piv = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        pv = M[c][c]
        M[c] = [v / pv for v in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                fac = M[r][c]
                M[r] = [a - fac * b for a, b in zip(M[r], M[c])]
    return [M[i][n] for i in range(n)]


def exact_monomial(u, v, w, l, m, n):
    return Fraction(u) ** l * Fraction(v) ** m * Fraction(w) ** n / (math.factorial(l) * math.factorial(m) * math.factorial(n))


def geometric_groups(x, y, z, depth, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)):
    """Recursive partition of point indices by comparing with node centres (upper
    child on the plane), the octant route of Alg. 1.  Returns {(level, path): set(idx)}."""
    out = {}

    def rec(idx, level, path, c, h):
        out[(level, path)] = set(idx.tolist())
        if level == depth or idx.size == 0:
            return
        bx = x[idx] >= c[0]
        by = y[idx] >= c[1]
        bz = z[idx] >= c[2]
        for o in range(8):
            sel = idx[(bx == bool(o & 4)) & (by == bool(o & 2)) & (bz == bool(o & 1))]
            if sel.size:
                cc = [c[a] + (0.25 if (o >> (2 - a)) & 1 else -0.25) * h[a] for a in range(3)]
                rec(sel, level + 1, path + (o,), cc, [hh / 2 for hh in h])

    h0 = [hi[a] - lo[a] for a in range(3)]
    rec(np.arange(len(x)), 0, (), [lo[a] + 0.5 * h0[a] for a in range(3)], h0)
    return out


# ----------------------------------------------------------------------------
# basis
# ----------------------------------------------------------------------------
def pin_basis_sizes():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "basis_sizes.txt")) if l.strip() and not l.startswith("#")]
    for order, size in rows:
        assert oracle.basis_size(int(order)) == int(size), (order, size)
    for p in range(0, 15):
        assert oracle.basis_size(p) == len(brute_monomials(p))


def test_basis_sizes_printed():
    pin_basis_sizes()


def pin_graded_order():
    for p in range(0, 9):
        ex = oracle.exponents(p)
        assert len(ex) == len(set(ex)) == oracle.basis_size(p)
        assert set(ex) == brute_monomials(p)
        degs = [sum(e) for e in ex]
        assert degs == sorted(degs)
        for k in range(p + 1):
            # the rank stride is the index of the first monomial of degree k
            assert degs.index(k) == k * (k + 1) * (k + 2) // 6
        if p >= 1:
            assert ex[1:4] == [(1, 0, 0), (0, 1, 0), (0, 0, 1)]


def test_graded_order_and_rank_stride():
    pin_graded_order()


def pin_moments_exact():
    rng = np.random.default_rng(7)
    u = rng.uniform(-1, 1, 5)
    v = rng.uniform(-1, 1, 5)
    w = rng.uniform(-1, 1, 5)
    for p in (0, 1, 3, 6):
        lam = oracle.moments(u, v, w, p)
        for j, (l, m, n) in enumerate(oracle.exponents(p)):
            for i in range(5):
                ex = float(exact_monomial(u[i], v[i], w[i], l, m, n))
                assert abs(lam[i, j] - ex) <= 4 * np.finfo(float).eps * max(abs(ex), 1e-300), (p, j, i)


def test_moments_exact():
    pin_moments_exact()


# ----------------------------------------------------------------------------
# keys and the octant partition
# ----------------------------------------------------------------------------
def adversarial_points(depth, seed=3):
    rng = np.random.default_rng(seed)
    h = 2.0 ** -depth
    n = 600
    x, y, z = rng.uniform(0, 1, (3, n))
    # points exactly on split planes at every level and on the box faces
    k = rng.integers(0, 2 ** depth + 1, (3, 200))
    pl = (k * h).clip(0, 1)
    x = np.concatenate([x, pl[0], [0.0, 1.0, 1.0, 0.5, 0.5, 0.25]])
    y = np.concatenate([y, pl[1], [0.0, 1.0, 0.0, 0.5, 0.5, 0.75]])
    z = np.concatenate([z, pl[2], [0.0, 1.0, 1.0, 0.5, 0.0, 0.125]])
    return x, y, z


def pin_morton_matches_geometric(depth=4):
    x, y, z = adversarial_points(depth)
    keys = oracle.morton(oracle.quantise(x, 0, 1, depth), oracle.quantise(y, 0, 1, depth),
                         oracle.quantise(z, 0, 1, depth), depth)
    groups = geometric_groups(x, y, z, depth)
    for (level, path), idx in groups.items():
        pre = 0
        for o in path:
            pre = (pre << 3) | o
        mine = set(np.nonzero((keys >> (3 * (depth - level))) == pre)[0].tolist())
        assert mine == idx, (level, path)


def test_morton_matches_geometric_partition():
    pin_morton_matches_geometric(4)
    pin_morton_matches_geometric(1)


def test_morton_hand_built():
    # one point in each octant of the unit cube: key = 4*bx + 2*by + bz
    pts = [(0.25 + 0.5 * ((o >> 2) & 1), 0.25 + 0.5 * ((o >> 1) & 1), 0.25 + 0.5 * (o & 1)) for o in range(8)]
    x, y, z = (np.array(a) for a in zip(*pts))
    keys = oracle.morton(oracle.quantise(x, 0, 1, 1), oracle.quantise(y, 0, 1, 1), oracle.quantise(z, 0, 1, 1), 1)
    assert keys.tolist() == list(range(8))
    # depth 2: the point (0.6, 0.1, 0.9): cells (2, 0, 3) -> bits x=10, y=00, z=11 -> (1,0,1),(0,0,1)
    k = oracle.morton(oracle.quantise(np.array([0.6]), 0, 1, 2), oracle.quantise(np.array([0.1]), 0, 1, 2),
                      oracle.quantise(np.array([0.9]), 0, 1, 2), 2)
    assert int(k[0]) == (0b101 << 3) | 0b001
    # x = hi goes to the last cell, x = lo to the first
    assert oracle.quantise(np.array([1.0, 0.0]), 0, 1, 3).tolist() == [7, 0]


# ----------------------------------------------------------------------------
# per-node least squares (Alg. 2)
# ----------------------------------------------------------------------------
def pin_exact_rational_ls():
    rng = np.random.default_rng(11)
    for p, n in ((1, 9), (2, 16), (3, 30)):
        u, v, w = (rng.uniform(-1, 1, n) for _ in range(3))
        r = rng.uniform(-1, 1, n)
        F, rd = fo.mesh_to_moments(u, v, w, r, p)
        assert not rd
        ex = oracle.exponents(p)
        rows = [[exact_monomial(u[i], v[i], w[i], *e) for e in ex] for i in range(n)]
        Fx = exact_lstsq(rows, [Fraction(t) for t in r])
        Fx = np.array([float(t) for t in Fx])
        lam = oracle.moments(u, v, w, p)
        kappa = np.linalg.cond(lam)
        err = np.max(np.abs(F - Fx)) / max(np.max(np.abs(Fx)), 1e-300)
        assert err <= 50 * kappa * len(ex) * np.finfo(float).eps, (p, err, kappa)


def test_exact_rational_least_squares():
    pin_exact_rational_ls()


def test_matches_svd_lstsq():
    rng = np.random.default_rng(5)
    for p in (2, 4, 6):
        n = 5 * oracle.basis_size(p)
        u, v, w = (rng.uniform(-1, 1, n) for _ in range(3))
        r = np.sin(3 * u) * np.cos(2 * v) + w ** 3
        F, _ = fo.mesh_to_moments(u, v, w, r, p)
        lam = oracle.moments(u, v, w, p)
        Fs, *_ = np.linalg.lstsq(lam, r, rcond=None)
        assert np.max(np.abs(lam @ F - lam @ Fs)) < 1e-12


def test_streamed_qr_equals_single_block():
    rng = np.random.default_rng(9)
    p, n = 4, 3000
    u, v, w = (rng.uniform(-1, 1, n) for _ in range(3))
    r = np.exp(u * v) - w
    F1, _ = fo.mesh_to_moments(u, v, w, r, p, block=n)
    F2, _ = fo.mesh_to_moments(u, v, w, r, p, block=257)
    assert np.max(np.abs(F1 - F2)) < 1e-11 * np.max(np.abs(F1))


def pin_polynomial_reproduction(p=4, seed=21, n=2000, depth=3):
    """A degree <= p polynomial is reproduced at the root: residual at rounding
    level, no child activates, and F holds the node-frame Taylor coefficients
    d^alpha f(c) (h/2)^|alpha| (since Lambda_alpha = u^alpha / alpha!)."""
    poly = random_poly(p, seed)
    x, y, z = synthetic.uniform_points(n, seed)
    f = poly_eval(poly, x, y, z)
    t = oracle.fit(x, y, z, f, p, 1e-11, depth)
    assert t.nodes == 1
    assert oracle.rms(t.residual) < 1e-13 * max(1.0, oracle.rms(f))
    c = (0.5, 0.5, 0.5)
    half = 0.5
    for j, e in enumerate(oracle.exponents(p)):
        want = poly_derivative_at(poly, e, c) * half ** sum(e)
        assert abs(t.coeffs[0, j] - want) < 1e-11, (e, t.coeffs[0, j], want)


def test_polynomial_reproduction():
    pin_polynomial_reproduction(4, 21)
    pin_polynomial_reproduction(6, 22, n=3000)
    pin_polynomial_reproduction(1, 23, n=50)


def pin_resolution_of_identity(p=5, seed=31):
    """Fit on grid p, evaluate on a disjoint grid q: a degree <= p polynomial
    is transformed exactly (the pointwise resolution of identity)."""
    poly = random_poly(p, seed)
    x, y, z = synthetic.uniform_points(1500, seed)
    qx, qy, qz = synthetic.uniform_points(1000, seed + 1)
    t = oracle.fit(x, y, z, poly_eval(poly, x, y, z), p, 1e-11, 3)
    got = oracle.evaluate(t, qx, qy, qz)
    assert oracle.max_abs(got - poly_eval(poly, qx, qy, qz)) < 1e-12


def test_resolution_of_identity():
    pin_resolution_of_identity()


# ----------------------------------------------------------------------------
# invariants of the decomposition (Alg. 1)
# ----------------------------------------------------------------------------
def pin_projection_orthogonality():
    """At a leaf, the final residual is the node's LS residual: Lambda^T r = 0."""
    pr = synthetic.small_problem(6000, 3, seed=41, tol=1e-9, depth=2)
    t = oracle.fit(pr.x, pr.y, pr.z, pr.f, pr.p, pr.tol, pr.max_depth)
    parents = {(int(l) - 1, int(pf) >> 3) for l, pf in zip(t.level, t.prefix) if l > 0}
    checked = 0
    for i in range(t.nodes):
        if (int(t.level[i]), int(t.prefix[i])) in parents:
            continue
        idx = t.order[t.begin[i]:t.begin[i] + t.count[i]]
        cell = fo._prefix_cell(int(t.prefix[i]), int(t.level[i]))
        c, s = oracle.node_frame(int(t.level[i]), cell, t.lo, t.hi)
        lam = oracle.moments((pr.x[idx] - c[0]) * s[0], (pr.y[idx] - c[1]) * s[1], (pr.z[idx] - c[2]) * s[2], pr.p)
        g = lam.T @ t.residual[idx]
        assert np.max(np.abs(g)) <= 1e-12 * np.linalg.norm(lam) * max(np.linalg.norm(t.residual[idx]), 1e-300) * 10
        checked += 1
    assert checked >= 8


def test_projection_orthogonality():
    pin_projection_orthogonality()


def pin_monotone_residual():
    pr = synthetic.small_problem(20000, 2, seed=43, tol=0.0, depth=4)
    prev = float(np.sum(pr.f.astype(np.float64) ** 2))
    for D in range(0, 5):
        t = oracle.fit(pr.x, pr.y, pr.z, pr.f, pr.p, 0.0, D)
        ss = float(np.sum(t.residual ** 2))
        assert ss <= prev * (1 + 1e-12), (D, ss, prev)
        prev = ss


def test_monotone_residual_by_depth():
    pin_monotone_residual()


def pin_mean_hierarchy():
    """p = 0: every node's coefficient is the mean of the residual it inherits."""
    pr = synthetic.small_problem(3000, 0, seed=47, tol=0.0, depth=3)
    t = oracle.fit(pr.x, pr.y, pr.z, pr.f, 0, 0.0, 3)
    D = 3
    keys = t.keys
    r = pr.f.astype(np.float64).copy()
    look = t.lookup()
    for d in range(D + 1):
        for pre in np.unique(keys >> (3 * (D - d))):
            if (d, int(pre)) not in look:
                continue
            sel = (keys >> (3 * (D - d))) == pre
            m = float(np.mean(r[sel]))
            assert abs(t.coeffs[look[(d, int(pre))], 0] - m) < 1e-14
            r[sel] -= m
    assert np.max(np.abs(r - t.residual)) < 1e-14


def test_p0_is_hierarchy_of_means():
    pin_mean_hierarchy()


def test_interpolation_when_n_equals_L():
    p = 3
    L = oracle.basis_size(p)
    rng = np.random.default_rng(53)
    x, y, z = rng.uniform(0, 1, (3, L))
    f = np.cos(5 * x) + y * z
    t = oracle.fit(x, y, z, f, p, 0.0, 3)
    assert t.nodes == 1
    assert oracle.max_abs(t.residual) < 1e-9


def test_p1_is_linear_regression():
    pr = synthetic.small_problem(500, 1, seed=59, tol=0.0, depth=0)
    t = oracle.fit(pr.x, pr.y, pr.z, pr.f, 1, 0.0, 0)
    X = np.stack([pr.x, pr.y, pr.z], 1).astype(np.float64)
    xm = X.mean(0)
    fm = pr.f.mean()
    beta = np.linalg.solve((X - xm).T @ (X - xm), (X - xm).T @ (pr.f - fm))
    fit_lr = fm + (X - xm) @ beta
    assert oracle.max_abs((pr.f - t.residual) - fit_lr) < 1e-13


def test_eval_at_points_equals_fitted_values():
    pr = synthetic.small_problem(8000, 3, seed=61, tol=1e-6, depth=3)
    t = oracle.fit(pr.x, pr.y, pr.z, pr.f, pr.p, pr.tol, pr.max_depth)
    assert t.nodes > 9
    got = oracle.evaluate(t, pr.x, pr.y, pr.z)
    assert oracle.max_abs(got - (pr.f - t.residual)) < 1e-13


def test_projection_is_idempotent():
    pr = synthetic.small_problem(2000, 4, seed=67, tol=0.0, depth=0)
    t = oracle.fit(pr.x, pr.y, pr.z, pr.f, 4, 0.0, 0)
    g = pr.f - t.residual
    t2 = oracle.fit(pr.x, pr.y, pr.z, g, 4, 0.0, 0)
    assert oracle.max_abs(t2.residual) < 1e-13


def test_termination_rules():
    pr = synthetic.small_problem(6000, 2, seed=71, tol=1e-4, depth=3)
    L = oracle.basis_size(2)
    t = oracle.fit(pr.x, pr.y, pr.z, pr.f, 2, 1e-4, 3)
    look = t.lookup()
    assert np.all(t.count >= L)
    assert np.all(t.level <= 3)
    for (d, pre) in look:
        if d > 0:
            assert (d - 1, pre >> 3) in look
    # every octant decision: a child exists iff E_RMS > tau (with n_o >= calL)
    for (d, pre, n_o, e) in t.decisions:
        assert n_o >= L
        assert ((d, pre) in look) == (e > 1e-4)
    # root only when the tolerance is huge or the depth cap is 0
    assert oracle.fit(pr.x, pr.y, pr.z, pr.f, 2, 1e9, 3).nodes == 1
    assert oracle.fit(pr.x, pr.y, pr.z, pr.f, 2, 0.0, 0).nodes == 1
    # tol = 0 with a depth cap: every octant with n_o >= calL is refined
    t0 = oracle.fit(pr.x, pr.y, pr.z, pr.f, 2, 0.0, 2)
    keys = t0.keys
    for d in (1, 2):
        pres, cnt = np.unique(keys >> (3 * (2 - d)), return_counts=True)
        want = {int(a) for a, c in zip(pres, cnt) if c >= L}
        got = {int(pf) for l, pf in zip(t0.level, t0.prefix) if l == d}
        # a child can only exist under an existing parent
        want = {w for w in want if d == 1 or (d - 1, w >> 3) in t0.lookup()}
        assert got == want


def test_rejects_bad_inputs():
    x, y, z = synthetic.uniform_points(100, 1)
    with pytest.raises(ValueError):
        oracle.fit(x[:19], y[:19], z[:19], x[:19], 3, 0.0, 2)   # n < calL = 20
    x2 = x.copy()
    x2[3] = 1.5
    with pytest.raises(ValueError):
        oracle.fit(x2, y, z, x, 1, 0.0, 2)
    x2[3] = np.nan
    with pytest.raises(ValueError):
        oracle.fit(x2, y, z, x, 1, 0.0, 2)


def test_rank_deficient_node_fitted_values_unique():
    # all points on the plane z = 0.5: the z-dependent monomials are dependent
    rng = np.random.default_rng(73)
    n = 400
    x, y = rng.uniform(0, 1, (2, n))
    z = np.full(n, 0.5)
    f = np.sin(4 * x) + y ** 2
    t = oracle.fit(x, y, z, f, 3, 0.0, 0)
    assert t.rank_deficient[0]
    # 2-D least squares with the 10 monomials x^a y^b, a+b <= 3 gives the same fit
    A = np.stack([x ** a * y ** b for a in range(4) for b in range(4 - a)], 1)
    c, *_ = np.linalg.lstsq(A, f, rcond=None)
    assert oracle.max_abs((f - t.residual) - A @ c) < 1e-12


# ----------------------------------------------------------------------------
# end-to-end magnitude on the paper's test function (soft pin)
# ----------------------------------------------------------------------------
@pytest.mark.slow
def test_franke_error_falls_with_order():
    x, y, z = synthetic.uniform_points(8 ** 4, 81)
    qx, qy, qz = synthetic.uniform_points(4000, 82)
    f = synthetic.franke3d(x, y, z)
    ft = synthetic.franke3d(qx, qy, qz)
    errs = []
    for p in (2, 4, 6):
        t = oracle.fit(x, y, z, f, p, 0.0, 0)
        errs.append(oracle.rms(oracle.evaluate(t, qx, qy, qz) - ft))
    assert errs[0] > errs[1] > errs[2]


# ----------------------------------------------------------------------------
# fixed-topology transform (the node set of a fitted tree, new values)
# ----------------------------------------------------------------------------
def _split_tree(seed=41):
    pr = synthetic.small_problem(6000, 3, seed=seed, tol=1e-9, depth=3)
    return pr, oracle.fit(pr.x, pr.y, pr.z, pr.f, pr.p, pr.tol, pr.max_depth)


def pin_fixed_topology_reproduces_fit():
    """Refitting the values a tree was built from walks the same nodes with the
    same residuals as Alg. 1 did: identical coefficients and residual."""
    pr, t = _split_tree()
    assert t.nodes > 9
    t2 = oracle.fit_fixed(t, pr.x, pr.y, pr.z, pr.f)
    np.testing.assert_array_equal(t2.coeffs, t.coeffs)
    np.testing.assert_array_equal(t2.residual, t.residual)


def test_fixed_topology_reproduces_fit():
    pin_fixed_topology_reproduces_fit()


def pin_fixed_topology_polynomial():
    """A degree <= p field on a tree built from other values: the root takes
    the node-frame Taylor coefficients, every other node ~0, the residual
    vanishes, and the node set is kept although this field would not split."""
    pr, t = _split_tree()
    poly = random_poly(pr.p, 5)
    f2 = poly_eval(poly, pr.x, pr.y, pr.z)
    t2 = oracle.fit_fixed(t, pr.x, pr.y, pr.z, f2)
    assert t2.nodes == t.nodes
    for j, e in enumerate(oracle.exponents(pr.p)):
        want = poly_derivative_at(poly, e, (0.5, 0.5, 0.5)) * 0.5 ** sum(e)
        assert abs(t2.coeffs[0, j] - want) < 1e-11, (e, t2.coeffs[0, j], want)
    assert np.max(np.abs(t2.coeffs[1:])) < 1e-10
    assert oracle.max_abs(t2.residual) < 1e-12


def test_fixed_topology_polynomial():
    pin_fixed_topology_polynomial()


def pin_fixed_topology_linear_and_orthogonal():
    """The fixed-topology map is linear in the values, and at every leaf the
    final residual of any field is orthogonal to the basis (Lambda^T r = 0)."""
    pr, t = _split_tree()
    rng = np.random.default_rng(7)
    f1 = rng.standard_normal(pr.n)
    f2 = np.sin(7 * pr.x) * pr.y
    a = oracle.fit_fixed(t, pr.x, pr.y, pr.z, f1)
    b = oracle.fit_fixed(t, pr.x, pr.y, pr.z, f2)
    c = oracle.fit_fixed(t, pr.x, pr.y, pr.z, 2.0 * f1 - 3.0 * f2)
    scale = np.max(np.abs(2.0 * a.coeffs)) + np.max(np.abs(3.0 * b.coeffs))
    assert np.max(np.abs(c.coeffs - (2.0 * a.coeffs - 3.0 * b.coeffs))) < 1e-12 * scale
    parents = {(int(l) - 1, int(pf) >> 3) for l, pf in zip(t.level, t.prefix) if l > 0}
    leaves = 0
    for i in range(t.nodes):
        if (int(t.level[i]), int(t.prefix[i])) in parents:
            continue
        idx = t.order[t.begin[i]:t.begin[i] + t.count[i]]
        cell = fo._prefix_cell(int(t.prefix[i]), int(t.level[i]))
        cc, s = oracle.node_frame(int(t.level[i]), cell, t.lo, t.hi)
        lam = oracle.moments((pr.x[idx] - cc[0]) * s[0], (pr.y[idx] - cc[1]) * s[1], (pr.z[idx] - cc[2]) * s[2],
                             pr.p)
        g = lam.T @ a.residual[idx]
        # rounding is relative to the values the node's fits started from
        assert np.max(np.abs(g)) <= 1e-11 * np.linalg.norm(lam) * np.linalg.norm(f1[idx])
        leaves += 1
    assert leaves >= 8


def test_fixed_topology_linear_and_orthogonal():
    pin_fixed_topology_linear_and_orthogonal()


def test_fixed_topology_rejects_other_points():
    pr, t = _split_tree()
    x = pr.x.copy()
    x[0] = 1.0 - x[0]
    with pytest.raises(ValueError):
        oracle.fit_fixed(t, x, pr.y, pr.z, pr.f)
    with pytest.raises(ValueError):
        oracle.fit_fixed(t, pr.x[:-1], pr.y[:-1], pr.z[:-1], pr.f[:-1])


# ----------------------------------------------------------------------------
# Gaussian-RBF factorisation (Section 2, eq. fullyfactored)
# ----------------------------------------------------------------------------
def pin_hermite_numbers():
    # H_n(0) from the polynomials themselves: H_0 = 1, H_2 = 4t^2 - 2,
    # H_4 = 16t^4 - 48t^2 + 12, H_6 = 64t^6 - 480t^4 + 720t^2 - 120 (textbook
    # recurrence H_{n+1} = 2t H_n - 2n H_{n-1}); He likewise (He_{n+1} = t He_n - n He_{n-1})
    H = {0: np.poly1d([1.0]), 1: np.poly1d([2.0, 0.0])}
    He = {0: np.poly1d([1.0]), 1: np.poly1d([1.0, 0.0])}
    t = np.poly1d([1.0, 0.0])
    for n in range(1, 14):
        H[n + 1] = 2 * t * H[n] - 2 * n * H[n - 1]
        He[n + 1] = t * He[n] - n * He[n - 1]
    for n in range(15):
        assert oracle.hermite_at_zero(n) == H[n](0.0)
        assert oracle.hermite_at_zero(n, "probabilists") == He[n](0.0)
    assert [oracle.hermite_at_zero(n) for n in (0, 2, 4, 6)] == [1.0, -2.0, 12.0, -120.0]


def pin_rbf_factored_converges_to_the_gaussian():
    # the truncated factorisation against exp(-eps^2 |x - x'|^2) evaluated
    # directly: the error falls with the order and reaches rounding level
    rng = np.random.default_rng(71)
    x, y, z = rng.uniform(-1, 1, (3, 40))
    xq, yq, zq = rng.uniform(-1, 1, (3, 30))
    d2 = (xq[:, None] - x[None, :]) ** 2 + (yq[:, None] - y[None, :]) ** 2 + (zq[:, None] - z[None, :]) ** 2
    for kind, scale in (("physicists", 1.0), ("probabilists", 0.5)):
        eps = 0.15
        direct = np.exp(-scale * eps * eps * d2)
        errs = [np.max(np.abs(oracle.rbf_factored(x, y, z, xq, yq, zq, p, eps, kind) - direct)) for p in (2, 6, 10, 14)]
        assert errs[0] > errs[1] > errs[2], (kind, errs)
        assert errs[3] < 1e-12, (kind, errs)


def pin_rbf_T_structure():
    T = oracle.rbf_T(6)
    assert np.array_equal(T, T.T)              # symmetric: h_n(0) vanishes for odd n
    assert T[0, 0] == 1.0
    ex = oracle.exponents(6)
    i = ex.index((2, 0, 0))
    assert T[i, 0] == -2.0 and T[0, i] == -2.0   # H_2(0)
    j = ex.index((1, 0, 0))
    assert T[j, j] == -(-2.0)                    # (-1)^1 H_2(0) H_0 H_0
    assert T[j, 0] == 0.0                        # H_1(0) = 0


def test_hermite_numbers():
    pin_hermite_numbers()


def test_rbf_factored_converges_to_the_gaussian():
    pin_rbf_factored_converges_to_the_gaussian()


def test_rbf_T_structure():
    pin_rbf_T_structure()


# ----------------------------------------------------------------------------
# mutation tests: a planted mistake in the oracle must fail a pin
# ----------------------------------------------------------------------------
def _mutant_moments_no_factorial(u, v, w, p):
    u, v, w = (np.asarray(a, dtype=np.float64) for a in (u, v, w))
    return np.stack([u ** l * v ** m * w ** n for (l, m, n) in fo.exponents(p)], 1)


def _mutant_exponents_lex(p):
    return [(l, m, n) for l in range(p + 1) for m in range(p + 1 - l) for n in range(p + 1 - l - m)]


def _mutant_basis_size(p):
    return fo.rank_stride(p)


def _mutant_morton_yx(qx, qy, qz, depth):
    key = np.zeros(np.shape(qx), dtype=np.int64)
    for b in range(depth - 1, -1, -1):
        key = (key << 3) | (((qy >> b) & 1) << 2) | (((qx >> b) & 1) << 1) | ((qz >> b) & 1)
    return key


def _mutant_frame_full_width(level, cell, lo, hi):
    c, s = _orig_frame(level, cell, lo, hi)
    return c, s / 2.0


def _mutant_residual_sign(u, v, w, r, F, p, block=fo.QR_BLOCK_ROWS):
    return np.asarray(r, dtype=np.float64) + fo.moments(u, v, w, p) @ F


def _mutant_drop_last_block(u, v, w, r, p, block=fo.QR_BLOCK_ROWS):
    n = u.shape[0]
    keep = max(fo.basis_size(p), n - n // 7)
    return _orig_mtm(u[:keep], v[:keep], w[:keep], r[:keep], p, block)


def _mutant_hermite_probabilists(n, kind="physicists"):
    return _orig_hermite(n, "probabilists")


def _mutant_rbf_T_no_sign(p, kind="physicists"):
    ex = fo.exponents(p)
    return np.abs(_orig_rbf_T(p, kind)) * np.array([[1.0 if (a + b + c) % 2 == 0 else 1.0 for _ in ex]
                                                      for (a, b, c) in ex])


def _mutant_fit_fixed_children_first(tree, x, y, z, f):
    rev = np.arange(tree.nodes)[::-1]
    t = fo.dataclasses.replace(tree, level=tree.level[rev], prefix=tree.prefix[rev], begin=tree.begin[rev],
                               count=tree.count[rev], coeffs=tree.coeffs[rev])
    out = _orig_fit_fixed(t, x, y, z, f)
    return fo.dataclasses.replace(tree, coeffs=out.coeffs[rev], residual=out.residual)


_orig_frame = fo.node_frame
_orig_mtm = fo.mesh_to_moments
_orig_fit_fixed = fo.fit_fixed
_orig_hermite = fo.hermite_at_zero
_orig_rbf_T = fo.rbf_T

MUTANTS = [
    ("moments", _mutant_moments_no_factorial),
    ("exponents", _mutant_exponents_lex),
    ("basis_size", _mutant_basis_size),
    ("morton", _mutant_morton_yx),
    ("node_frame", _mutant_frame_full_width),
    ("residual_update", _mutant_residual_sign),
    ("mesh_to_moments", _mutant_drop_last_block),
    ("fit_fixed", _mutant_fit_fixed_children_first),
    ("hermite_at_zero", _mutant_hermite_probabilists),
    ("rbf_T", _mutant_rbf_T_no_sign),
]

PINS = [pin_basis_sizes, pin_graded_order, pin_moments_exact, pin_morton_matches_geometric,
        pin_exact_rational_ls, pin_polynomial_reproduction, pin_resolution_of_identity,
        pin_projection_orthogonality, pin_monotone_residual, pin_mean_hierarchy,
        pin_fixed_topology_reproduces_fit, pin_fixed_topology_polynomial, pin_fixed_topology_linear_and_orthogonal,
        pin_hermite_numbers, pin_rbf_factored_converges_to_the_gaussian, pin_rbf_T_structure]


@pytest.mark.parametrize("name,mutant", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(monkeypatch, name, mutant):
    monkeypatch.setattr(fo, name, mutant)
    if hasattr(oracle, name):
        monkeypatch.setattr(oracle, name, mutant)
    failed = []
    for pin in PINS:
        try:
            pin()
        except (AssertionError, ValueError, IndexError, np.linalg.LinAlgError):
            failed.append(pin.__name__)
    assert failed, f"no pin caught the planted mistake in {name}"
