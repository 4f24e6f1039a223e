"""Plain FP64 CPU oracle of the free-mesh transform (FMT): fit and evaluation.

TEST INFRASTRUCTURE.  This module exists to check the GPU library, never to
serve results: only the test suite, the package smoke check and the CPU
baseline leg of the benchmark may import or call it.  It shares no code with
the GPU path (no kernels, tables, constants or helpers); the only module both
sides use is ``synthetic``, which draws inputs and holds none of the method.

What is computed (all arithmetic IEEE float64; float32 inputs promoted exactly):

* Basis (Section 2, the geometric moments and the rank stride): exponents
  alpha = (l, m, n) with l+m+n <= p in graded order (degree 0, then the three
  degree-1 monomials x, y, z, ...), so the first index of degree k is the rank
  stride k(k+1)(k+2)/6, and Lambda_alpha(u) = u^l v^m w^n / (l! m! n!).  The
  basis size is calL = (p+1)(p+2)(p+3)/6; this is the reading that reproduces
  the printed sizes 84, 286, 680 for orders 6, 10, 14 (Section 3).
* Alg. 1 (recursive octree decomposition of the residual): at a node, move the
  node's points into the node frame u = (x - c) * (2/h) in [-1, 1]^3, fit the
  residual there (Alg. 2), order the points by octant, and descend into an
  octant o only if it holds n_o >= calL points, the depth cap allows it, and the
  octant's RMS residual sqrt(sum r^2 / n_o) exceeds tau (strict).  The root is
  always fitted.
* Alg. 2 (moments of one node): build the Vandermonde matrix Lambda of the
  node's points, Householder-QR it (LAPACK dgeqrf through numpy), form
  F = R^{-1} Q^T r, and subtract Lambda F from the residual.  Q^T r is read off
  the QR of the augmented matrix [Lambda | r] (its last column), which is the
  same Householder process without forming Q; tall nodes are factored in row
  blocks and the stacked triangles re-factored (a streamed QR), so memory stays
  O(calL^2) per block.  A numerically rank-deficient R -- condition number of
  the column-equilibrated triangle above 1/(1e3 eps), e.g. coplanar points on
  a clipped face -- is solved in the minimum-norm sense instead (the fitted
  values stay unique).
* Octants are taken from the integer cell of each point at the finest depth D:
  q = clamp(floor((x - lo) * (2^D / (hi - lo))), 0, 2^D - 1) per axis, and the
  octant at depth d+1 is the three bits (x highest) of the cells at that depth.
  A point on a split plane goes to the upper octant; a point at x = hi goes to
  the last cell.
* Fixed-topology transform (the operator I' of Section 2, eq. identityprime, with the node set
  held fixed): for new values f on the same points, Alg. 2 at every node of an
  existing tree, parents before children, each node fitting the residual its
  ancestors left; no octant test is taken, so the map f -> coefficients is
  linear.
* Gaussian-RBF factorisation (Section 2, eq. fullyfactored): the kernel
  phi(|x' - x|) = exp(-eps^2 |x' - x|^2) expanded in Taylor series and
  truncated to the calL monomials of degree <= p on each side,
  phi ~ Lambda(x) . E . T . E . Lambda(x')^T with E = diag(eps^|alpha|) and
  T_ab = (-1)^|a| h_{a1+b1}(0) h_{a2+b2}(0) h_{a3+b3}(0), the h_n(0) being the
  values at zero of the Hermite functions h_n(t) = exp(-t^2) H_n(t) that the
  section defines (physicists' Hermite polynomials: H_n(0) = (-1)^(n/2)
  n!/(n/2)! for even n, 0 for odd n).  The section's printed closed form
  (-1)^(n/2) (n-1)!! is the probabilists' He_n(0), which expands
  exp(-eps^2 |x' - x|^2 / 2) instead; both are available.
* Evaluation (the practical form f'_q = Lambda'_q F_p of Section 2, summed over
  the tree as the residual decomposition implies): for a query, walk from the
  root down while the node holding the query's cell exists, adding each node's
  Lambda(u_node(q)) . F_node.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import scipy.linalg

__all__ = [
    "rank_stride", "basis_size", "exponents", "moments",
    "quantise", "morton", "node_frame", "mesh_to_moments",
    "Tree", "fit", "fit_fixed", "evaluate", "rms", "max_abs",
    "hermite_at_zero", "rbf_T", "rbf_factored",
]

EPS = np.finfo(np.float64).eps
QR_BLOCK_ROWS = 32768


# ----------------------------------------------------------------------------
# basis (Section 2: rank stride, geometric moments)
# ----------------------------------------------------------------------------
def rank_stride(i: int) -> int:
    """Number of 3-D monomials of degree < i: i(i+1)(i+2)/6."""
    return i * (i + 1) * (i + 2) // 6


def basis_size(p: int) -> int:
    """calL for maximum total degree p: all monomials of degree <= p."""
    return rank_stride(p + 1)


def exponents(p: int) -> List[Tuple[int, int, int]]:
    """Graded order: by degree k, then l descending, then m descending."""
    out = []
    for k in range(p + 1):
        for l in range(k, -1, -1):
            for m in range(k - l, -1, -1):
                out.append((l, m, k - l - m))
    return out


def moments(u, v, w, p: int) -> np.ndarray:
    """Vandermonde matrix of geometric moments, shape (n, calL)."""
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    cols = []
    for (l, m, n) in exponents(p):
        denom = float(math.factorial(l) * math.factorial(m) * math.factorial(n))
        cols.append((u ** l) * (v ** m) * (w ** n) / denom)
    return np.stack(cols, axis=1) if cols else np.zeros((u.shape[0], 0))


# ----------------------------------------------------------------------------
# keys and node geometry
# ----------------------------------------------------------------------------
def quantise(x, lo: float, hi: float, depth: int) -> np.ndarray:
    """Integer cell index at depth D along one axis (clamped to the box)."""
    x = np.asarray(x, dtype=np.float64)
    scale = float(2 ** depth) / (float(hi) - float(lo))
    q = np.floor((x - float(lo)) * scale)
    q = np.clip(q, 0, 2 ** depth - 1)
    return q.astype(np.int64)


def morton(qx, qy, qz, depth: int) -> np.ndarray:
    """Interleave cell bits: for each level from the top, (x, y, z) with x highest."""
    key = np.zeros(np.shape(qx), dtype=np.int64)
    for b in range(depth - 1, -1, -1):
        key = (key << 3) | (((qx >> b) & 1) << 2) | (((qy >> b) & 1) << 1) | ((qz >> b) & 1)
    return key


def node_frame(level: int, cell: Tuple[int, int, int], lo, hi):
    """Centre c and dilation s of a node so that u = (x - c) * s lies in [-1, 1]^3."""
    c = np.empty(3)
    s = np.empty(3)
    for a in range(3):
        h = (float(hi[a]) - float(lo[a])) / float(2 ** level)
        c[a] = float(lo[a]) + (cell[a] + 0.5) * h
        s[a] = 2.0 / h
    return c, s


# ----------------------------------------------------------------------------
# Alg. 2: least-squares moments of one node
# ----------------------------------------------------------------------------
def _qr_r(a: np.ndarray) -> np.ndarray:
    return np.linalg.qr(a, mode="r")


def mesh_to_moments(u, v, w, r, p: int, block: int = QR_BLOCK_ROWS):
    """Fit F minimising ||Lambda F - r||_2 by Householder QR; return (F, rank_deficient).

    The residual is *not* modified here; the caller subtracts Lambda F.
    """
    n = u.shape[0]
    L = basis_size(p)
    if n < L:
        raise ValueError("under-determined node: n < calL")
    tri = []
    colnorm2 = np.zeros(L)
    for s in range(0, n, block):
        e = min(n, s + block)
        lam = moments(u[s:e], v[s:e], w[s:e], p)
        colnorm2 += np.einsum("ij,ij->j", lam, lam)
        tri.append(_qr_r(np.column_stack([lam, r[s:e]])))
    R = tri[0] if len(tri) == 1 else _qr_r(np.vstack(tri))
    Rl = R[:L, :L]
    z = R[:L, L]
    # numerical rank: condition number of the column-equilibrated triangle
    scale = 1.0 / np.sqrt(np.maximum(colnorm2, np.finfo(np.float64).tiny))
    sv = np.linalg.svd(Rl * scale[None, :], compute_uv=False)
    rank_def = bool(sv[-1] <= 1e3 * EPS * sv[0])
    if not rank_def:
        F = scipy.linalg.solve_triangular(Rl, z, lower=False)
    else:
        G, *_ = np.linalg.lstsq(Rl * scale[None, :], z, rcond=1e3 * EPS)
        F = G * scale
    return F, rank_def


def residual_update(u, v, w, r, F, p: int, block: int = QR_BLOCK_ROWS) -> np.ndarray:
    """r - Lambda F, in row blocks."""
    out = np.array(r, dtype=np.float64, copy=True)
    for s in range(0, u.shape[0], block):
        e = min(u.shape[0], s + block)
        out[s:e] -= moments(u[s:e], v[s:e], w[s:e], p) @ F
    return out


# ----------------------------------------------------------------------------
# Alg. 1: the tree
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Tree:
    p: int
    tol: float
    max_depth: int
    lo: np.ndarray
    hi: np.ndarray
    # nodes in (level, prefix) order
    level: np.ndarray        # int
    prefix: np.ndarray       # int, key >> 3(D - level)
    begin: np.ndarray        # first position in the key-sorted point order
    count: np.ndarray        # points in the node
    coeffs: np.ndarray       # (nodes, calL) in graded order
    rank_deficient: np.ndarray
    margin: np.ndarray       # per node: E_RMS/tau - 1 of the decision that created it (nan for root)
    # per input point
    keys: np.ndarray
    order: np.ndarray        # key-sorted position -> input index (stable)
    residual: np.ndarray     # final residual, float64
    leaf: np.ndarray         # index of the deepest node holding the point
    # every octant decision taken (for tie reporting): (level, prefix, n_o, E_RMS)
    decisions: List[Tuple[int, int, int, float]]

    @property
    def L(self) -> int:
        return basis_size(self.p)

    @property
    def nodes(self) -> int:
        return int(self.level.shape[0])

    def lookup(self) -> Dict[Tuple[int, int], int]:
        return {(int(a), int(b)): i for i, (a, b) in enumerate(zip(self.level, self.prefix))}


def _cells(x, y, z, lo, hi, depth):
    return quantise(x, lo[0], hi[0], depth), quantise(y, lo[1], hi[1], depth), quantise(z, lo[2], hi[2], depth)


def fit(x, y, z, f, p: int, tol: float, max_depth: int,
        lo: Sequence[float] = (0.0, 0.0, 0.0), hi: Sequence[float] = (1.0, 1.0, 1.0)) -> Tree:
    """Alg. 1 from the root; returns the whole tree with per-point outputs."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    N = x.shape[0]
    L = basis_size(p)
    D = int(max_depth)
    if N < L:
        raise ValueError("under-determined root: N < calL")
    for a, arr in enumerate((x, y, z)):
        if not np.all(np.isfinite(arr)) or np.any(arr < lo[a]) or np.any(arr > hi[a]):
            raise ValueError("point outside the box")
    qx, qy, qz = _cells(x, y, z, lo, hi, D)
    keys = morton(qx, qy, qz, D)
    order = np.argsort(keys, kind="stable")
    sorted_keys = keys[order]

    r = f.copy()
    leaf = np.zeros(N, dtype=np.int64)
    found = []        # (level, prefix, count, F, rank_def, margin, idx)
    decisions = []

    def visit(idx: np.ndarray, level: int, cell: Tuple[int, int, int], margin: float):
        # coordinate transform into the node frame
        c, s = node_frame(level, cell, lo, hi)
        u = (x[idx] - c[0]) * s[0]
        v = (y[idx] - c[1]) * s[1]
        w = (z[idx] - c[2]) * s[2]
        # Alg. 2: moments, then residual update
        F, rdef = mesh_to_moments(u, v, w, r[idx], p)
        r[idx] = residual_update(u, v, w, r[idx], F, p)
        prefix = int(keys[idx[0]] >> (3 * (D - level)))
        found.append((level, prefix, idx.shape[0], F, rdef, margin, idx))
        if level == D:
            return
        # order by octant: the next bit of each axis' cell
        b = D - level - 1
        octs = (((qx[idx] >> b) & 1) << 2) | (((qy[idx] >> b) & 1) << 1) | ((qz[idx] >> b) & 1)
        for o in range(8):
            sel = idx[octs == o]
            n_o = sel.shape[0]
            if n_o < L:            # look-ahead on the point count first
                continue
            e_rms = math.sqrt(float(np.sum(r[sel] ** 2)) / n_o)
            decisions.append((level + 1, (prefix << 3) | o, n_o, e_rms))
            if e_rms > tol:
                child = (2 * cell[0] + ((o >> 2) & 1), 2 * cell[1] + ((o >> 1) & 1), 2 * cell[2] + (o & 1))
                visit(sel, level + 1, child, (e_rms / tol - 1.0) if tol > 0 else math.inf)

    visit(order.copy(), 0, (0, 0, 0), math.nan)

    found.sort(key=lambda t: (t[0], t[1]))
    level = np.array([t[0] for t in found], dtype=np.int64)
    prefix = np.array([t[1] for t in found], dtype=np.int64)
    count = np.array([t[2] for t in found], dtype=np.int64)
    coeffs = np.array([t[3] for t in found], dtype=np.float64).reshape(len(found), L)
    rdef = np.array([t[4] for t in found], dtype=bool)
    margin = np.array([t[5] for t in found], dtype=np.float64)
    begin = np.searchsorted(sorted_keys, prefix << (3 * (D - level)), side="left").astype(np.int64)
    for i, t in enumerate(found):       # deeper nodes overwrite shallower ones
        leaf[t[6]] = i
    return Tree(p=p, tol=float(tol), max_depth=D, lo=lo, hi=hi, level=level, prefix=prefix,
                begin=begin, count=count, coeffs=coeffs, rank_deficient=rdef, margin=margin,
                keys=keys, order=order, residual=r, leaf=leaf, decisions=decisions)


def fit_fixed(tree: Tree, x, y, z, f) -> Tree:
    """Alg. 2 at every node of `tree` for new values f on the tree's points.

    The node set, point ranges and frames are the tree's; nodes are taken in
    (level, prefix) order, so every node fits the residual left by all of its
    ancestors (siblings hold disjoint points, so this is the order Alg. 1's
    recursion produces for each node).  Returns a tree with the same topology
    and the new coefficients, rank flags and final residual.
    """
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    D = tree.max_depth
    if x.shape[0] != tree.keys.shape[0] or f.shape[0] != x.shape[0]:
        raise ValueError("the values must live on the tree's points")
    qx, qy, qz = _cells(x, y, z, tree.lo, tree.hi, D)
    if not np.array_equal(morton(qx, qy, qz, D), tree.keys):
        raise ValueError("the points differ from the tree's points")
    r = f.copy()
    coeffs = np.zeros_like(tree.coeffs)
    rdef = np.zeros(tree.nodes, dtype=bool)
    for i in range(tree.nodes):
        d = int(tree.level[i])
        idx = tree.order[tree.begin[i]:tree.begin[i] + tree.count[i]]
        c, s = node_frame(d, _prefix_cell(int(tree.prefix[i]), d), tree.lo, tree.hi)
        u = (x[idx] - c[0]) * s[0]
        v = (y[idx] - c[1]) * s[1]
        w = (z[idx] - c[2]) * s[2]
        F, rdef[i] = mesh_to_moments(u, v, w, r[idx], tree.p)
        r[idx] = residual_update(u, v, w, r[idx], F, tree.p)
        coeffs[i] = F
    return dataclasses.replace(tree, coeffs=coeffs, rank_deficient=rdef, residual=r, decisions=[])


def evaluate(tree: Tree, qx, qy, qz) -> np.ndarray:
    """Sum of Lambda(u_node(q)) . F_node over the existing ancestors of each query."""
    qx = np.asarray(qx, dtype=np.float64)
    qy = np.asarray(qy, dtype=np.float64)
    qz = np.asarray(qz, dtype=np.float64)
    D = tree.max_depth
    cx, cy, cz = _cells(qx, qy, qz, tree.lo, tree.hi, D)
    keys = morton(cx, cy, cz, D)
    order = np.argsort(keys, kind="stable")
    sk = keys[order]
    out = np.zeros(qx.shape[0])
    # a query is inside node (d, prefix) iff its key lies in that node's key range;
    # because a node exists only under an existing parent, summing over every node
    # whose key range holds the query is the root-to-leaf walk
    for i in range(tree.nodes):
        d = int(tree.level[i])
        pre = int(tree.prefix[i])
        a = np.searchsorted(sk, pre << (3 * (D - d)), side="left")
        b = np.searchsorted(sk, (pre + 1) << (3 * (D - d)), side="left")
        if b <= a:
            continue
        sel = order[a:b]
        cell = _prefix_cell(pre, d)
        c, s = node_frame(d, cell, tree.lo, tree.hi)
        lam = moments((qx[sel] - c[0]) * s[0], (qy[sel] - c[1]) * s[1], (qz[sel] - c[2]) * s[2], tree.p)
        out[sel] += lam @ tree.coeffs[i]
    return out


def _prefix_cell(prefix: int, level: int) -> Tuple[int, int, int]:
    i = j = k = 0
    for b in range(level):
        t = (prefix >> (3 * (level - 1 - b))) & 7
        i = (i << 1) | ((t >> 2) & 1)
        j = (j << 1) | ((t >> 1) & 1)
        k = (k << 1) | (t & 1)
    return i, j, k


# ----------------------------------------------------------------------------
# Gaussian-RBF factorisation (Section 2, eq. fullyfactored)
# ----------------------------------------------------------------------------
def hermite_at_zero(n: int, kind: str = "physicists") -> float:
    """h_n(0): the Hermite function exp(-t^2) H_n(t) at t = 0 (physicists'),
    or the probabilists' He_n(0) that the section prints."""
    if n % 2:
        return 0.0
    sign = -1.0 if (n // 2) % 2 else 1.0
    if kind == "physicists":
        return sign * float(math.factorial(n) // math.factorial(n // 2))
    if kind == "probabilists":
        dfact = 1
        for k in range(n - 1, 0, -2):
            dfact *= k
        return sign * float(dfact)
    raise ValueError("kind must be 'physicists' or 'probabilists'")


def rbf_T(p: int, kind: str = "physicists") -> np.ndarray:
    """T_ab = (-1)^|a| h_{a1+b1}(0) h_{a2+b2}(0) h_{a3+b3}(0) over the graded basis."""
    ex = exponents(p)
    L = len(ex)
    T = np.zeros((L, L))
    for i, (a1, a2, a3) in enumerate(ex):
        sg = -1.0 if (a1 + a2 + a3) % 2 else 1.0
        for j, (b1, b2, b3) in enumerate(ex):
            T[i, j] = sg * (hermite_at_zero(a1 + b1, kind) * hermite_at_zero(a2 + b2, kind)
                            * hermite_at_zero(a3 + b3, kind))
    return T


def rbf_factored(x, y, z, xq, yq, zq, p: int, eps: float, kind: str = "physicists") -> np.ndarray:
    """phi'_{q i} = Lambda(x_q) E T E Lambda(x_i)^T, shape (len(xq), len(x))."""
    E = np.array([float(eps) ** (a + b + c) for (a, b, c) in exponents(p)])
    C = E[:, None] * rbf_T(p, kind) * E[None, :]
    return moments(xq, yq, zq, p) @ C @ moments(x, y, z, p).T


def rms(a) -> float:
    a = np.asarray(a, dtype=np.float64)
    return float(np.sqrt(np.mean(a * a))) if a.size else 0.0


def max_abs(a) -> float:
    a = np.asarray(a, dtype=np.float64)
    return float(np.max(np.abs(a))) if a.size else 0.0
