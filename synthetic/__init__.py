"""Seeded synthetic workloads shaped like the paper's experiments.

This module only draws inputs: scattered points in the unit cube and sample
values of closed-form test functions at those points.  It holds none of the
interpolation method's arithmetic, so both the CPU oracle and the GPU path may
use it without sharing any code of the method.

The paper measures on random (quasi-uniform) grids in the unit cube with
closed-form values (Section "Free Mesh Transform"; the 3-D Franke function of
eq. (eqF1)).  The workloads below keep that shape: uniform or clustered
random points, values from a sum of anisotropic Gaussian bumps or from the
Franke function.

Recipe (every draw uses ``numpy.random.default_rng(seed)``, PCG64):
  * coordinates are drawn in float64, then rounded once to the storage dtype;
  * values are evaluated in float64 at the *rounded* coordinates, then rounded
    once to the storage dtype;
  * Gaussian-mixture points are clipped to the unit cube, so some lie exactly
    on a face.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

__all__ = [
    "Bumps", "draw_bumps", "bumps_value", "franke3d",
    "uniform_points", "mixture_points",
    "Problem", "config1", "config2", "config3", "config5", "small_problem",
    "request_stream",
]


# ----------------------------------------------------------------------------
# test functions
# ----------------------------------------------------------------------------
@dataclasses.dataclass(frozen=True)
class Bumps:
    """Sum of axis-aligned anisotropic Gaussians a*exp(-sum_d (x_d-c_d)^2/(2 w_d^2))."""
    centres: np.ndarray   # (k, 3)
    widths: np.ndarray    # (k, 3)
    amps: np.ndarray      # (k,)


def draw_bumps(seed: int, k: int = 4, wlo: float = 0.05, whi: float = 0.3) -> Bumps:
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, 1.0, size=(k, 3))
    widths = rng.uniform(wlo, whi, size=(k, 3))
    amps = rng.uniform(-1.0, 1.0, size=k)
    return Bumps(centres, widths, amps)


def bumps_value(b: Bumps, x, y, z) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    out = np.zeros_like(x)
    for c, w, a in zip(b.centres, b.widths, b.amps):
        e = ((x - c[0]) ** 2 / (2 * w[0] ** 2) + (y - c[1]) ** 2 / (2 * w[1] ** 2)
             + (z - c[2]) ** 2 / (2 * w[2] ** 2))
        out += a * np.exp(-e)
    return out


def franke3d(x, y, z) -> np.ndarray:
    """The 3-D Franke function as printed in eq. (eqF1) of the paper."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    t1 = np.exp(-0.25 * ((9 * x - 2) ** 2 + (9 * y - 2) ** 2 + (9 * z - 2) ** 2))
    t2 = np.exp(-((9 * x + 1) ** 2) / 49.0 - ((9 * y + 1) ** 2) / 10.0 - ((9 * z + 1) ** 2) / 10.0)
    t3 = np.exp(-0.25 * ((9 * x - 7) ** 2 + (9 * y - 3) ** 2 + (9 * z - 5) ** 2))
    t4 = np.exp(-((9 * x - 4) ** 2) - (9 * y - 7) ** 2 - (9 * z - 5) ** 2)
    return 0.75 * (t1 + t2) + 0.5 * t3 - 0.2 * t4


# ----------------------------------------------------------------------------
# point clouds
# ----------------------------------------------------------------------------
def uniform_points(n: int, seed: int, dtype=np.float64):
    rng = np.random.default_rng(seed)
    pts = rng.uniform(0.0, 1.0, size=(3, n)).astype(dtype)
    return pts[0].copy(), pts[1].copy(), pts[2].copy()


def mixture_points(n: int, seed: int, ncomp: int, slo: float = 0.02, shi: float = 0.2,
                   dtype=np.float64):
    """Equal-weight isotropic Gaussian mixture, centres U[0,1]^3, clipped to [0,1]^3."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, 1.0, size=(ncomp, 3))
    sig = rng.uniform(slo, shi, size=ncomp)
    comp = rng.integers(0, ncomp, size=n)
    pts = centres[comp].T + sig[comp][None, :] * rng.standard_normal(size=(3, n))
    pts = np.clip(pts, 0.0, 1.0).astype(dtype)
    return pts[0].copy(), pts[1].copy(), pts[2].copy()


# ----------------------------------------------------------------------------
# problems
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Problem:
    """One fit (and its queries): arrays in the storage dtype plus method parameters."""
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    f: np.ndarray
    p: int
    tol: float
    max_depth: int
    qx: Optional[np.ndarray] = None
    qy: Optional[np.ndarray] = None
    qz: Optional[np.ndarray] = None
    qf_true: Optional[np.ndarray] = None   # float64 truth at the (rounded) query points
    f_true: Optional[np.ndarray] = None    # float64 truth at the (rounded) points
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def dtype(self):
        return self.x.dtype


def _values(fun, x, y, z, dtype):
    ftrue = fun(x.astype(np.float64), y.astype(np.float64), z.astype(np.float64))
    return ftrue.astype(dtype), ftrue


def _make(name, x, y, z, fun, p, tol, depth, q=None, dtype=np.float64):
    f, ftrue = _values(fun, x, y, z, dtype)
    pr = Problem(x=x, y=y, z=z, f=f, p=p, tol=tol, max_depth=depth, f_true=ftrue, name=name)
    if q is not None:
        qx, qy, qz = q
        pr.qx, pr.qy, pr.qz = qx, qy, qz
        pr.qf_true = fun(qx.astype(np.float64), qy.astype(np.float64), qz.astype(np.float64))
    return pr


def scoping_problem(n: int, p: int, tol: float, seed: int, depth: int = 10) -> Problem:
    """The paper's scoping workload (Section 4): the 3-D Franke function on n
    uniform random points in [0,1]^3 (float64), evaluated on a separate random
    grid of the same size."""
    x, y, z = uniform_points(n, seed, np.float64)
    q = uniform_points(n, seed + 700, np.float64)
    return _make(f"scoping(n={n},p={p},tol={tol})", x, y, z, franke3d, p, tol, depth, q, np.float64)


def config1(seed: int = 1000) -> Problem:
    """N=4096 uniform, 4 bumps, p=4, uniform depth 3 (tol 0), 8192 queries, float64."""
    b = draw_bumps(seed + 500)
    x, y, z = uniform_points(4096, seed, np.float64)
    q = uniform_points(8192, seed + 700, np.float64)
    return _make("config1", x, y, z, lambda a, c, d: bumps_value(b, a, c, d), 4, 0.0, 3, q, np.float64)


def config2(seed: int = 2000, n: int = 1 << 20, nq: int = 1 << 22) -> Problem:
    """N=2^20 uniform (float32 storage), 4 bumps, p=6, depth<=6, tol 1e-8, 2^22 queries."""
    b = draw_bumps(seed + 500)
    x, y, z = uniform_points(n, seed, np.float32)
    q = uniform_points(nq, seed + 700, np.float32)
    return _make("config2", x, y, z, lambda a, c, d: bumps_value(b, a, c, d), 6, 1e-8, 6, q, np.float32)


def config3(seed0: int = 3000, count: int = 256, nlo: float = 1e3, nhi: float = 2e5,
            nq: int = 4096) -> List[Problem]:
    """Batched uneven problems: N log-uniform, 1-8 component mixtures, p in {4,5,6}."""
    rng = np.random.default_rng(seed0)
    ns = np.exp(rng.uniform(math.log(nlo), math.log(nhi), size=count)).astype(np.int64)
    ps = rng.integers(4, 7, size=count)
    comps = rng.integers(1, 9, size=count)
    out = []
    for k in range(count):
        s = seed0 + 1 + k
        b = draw_bumps(s + 100000)
        x, y, z = mixture_points(int(ns[k]), s, int(comps[k]), dtype=np.float32)
        q = mixture_points(nq, s + 200000, int(comps[k]), dtype=np.float32)
        out.append(_make(f"config3[{k}]", x, y, z, lambda a, c, d, b=b: bumps_value(b, a, c, d),
                         int(ps[k]), 1e-8, 6, q, np.float32))
    return out


def config5(seed: int = 5000, n: int = 1 << 26, nq: int = 1 << 26) -> Problem:
    """Large clustered fit: 32-component mixture (float32), p=8, depth<=10, tol 1e-8."""
    b = draw_bumps(seed + 500)
    x, y, z = mixture_points(n, seed, 32, dtype=np.float32)
    q = mixture_points(nq, seed + 700, 32, dtype=np.float32) if nq else None
    return _make("config5", x, y, z, lambda a, c, d: bumps_value(b, a, c, d), 8, 1e-8, 10, q, np.float32)


def small_problem(n: int, p: int, seed: int, tol: float = 1e-8, depth: int = 4,
                  dtype=np.float64, clustered: bool = False, nq: int = 0,
                  fun: str = "bumps") -> Problem:
    """A scaled-down instance of the same families for tests."""
    if clustered:
        x, y, z = mixture_points(n, seed, 4, dtype=dtype)
    else:
        x, y, z = uniform_points(n, seed, dtype)
    q = uniform_points(nq, seed + 700, dtype) if nq else None
    if fun == "franke":
        g = franke3d
    else:
        b = draw_bumps(seed + 500)
        g = lambda a, c, d: bumps_value(b, a, c, d)  # noqa: E731
    return _make(f"small(n={n},p={p},seed={seed})", x, y, z, g, p, tol, depth, q, dtype)


def request_stream(seed: int, count: int, fit_frac: float = 0.3, nq_lo: float = 1e4,
                   nq_hi: float = 1e6, n_lo: float = 1e3, n_hi: float = 1e6, p: int = 5,
                   qps: float = 100.0):
    """Poisson request stream for the serving workload.

    Returns a list of dicts {t, kind ('fit'|'eval'), n, seed, p}; arrays are drawn
    lazily by the consumer from ``seed`` so the stream itself stays small.
    """
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / qps, size=count))
    kinds = np.where(rng.uniform(size=count) < fit_frac, "fit", "eval")
    out = []
    for i in range(count):
        if kinds[i] == "fit":
            n = int(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi))))
        else:
            n = int(math.exp(rng.uniform(math.log(nq_lo), math.log(nq_hi))))
        out.append(dict(t=float(t[i]), kind=str(kinds[i]), n=n, seed=seed * 7919 + i, p=p,
                        ncomp=int(rng.integers(1, 9))))
    return out
