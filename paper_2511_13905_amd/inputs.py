"""Seeded synthetic problem generators.

These build the inputs of the projection subproblem (the linearized problem of
Sec. 3.2, eq. (linearized), and its regularized form, eq. (regularized_projection))
with the shapes, sizes and value distributions of the paper's four benchmark
classes (Sec. 4.1: volume-constrained compliance, compliance-constrained volume,
multi-material, volume + centre of mass).  The paper's own inputs come out of
an FEA run, which is out of scope; these are stand-ins of the same structure.

This module is shared by the tests, the benchmark and the smoke check.  It
contains no part of the solver: it draws random numbers, lays out grids and
forms right-hand sides.  The one place it evaluates the clip map is the recipe
that *plants* a right-hand side b from a chosen multiplier (b is an input of the
problem; the solver's job is the inverse direction).

All values are generated in float64 and rounded once to the stream dtype; the
rounded arrays are the problem.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

LO = 1e-3          # x_min of the box [x_min, 1]
HI = 1.0
C_DEFAULT = 1e12   # the paper's default penalty C (Sec. 3.5 defaults)


@dataclass
class Problem:
    """One projection instance: project y onto {lo <= x <= hi, A x <= b}.

    kind: "single" (m = 1, dense row), "independent" (m disjoint blocks, one
    coefficient per element in ``A`` of shape [n], block j owns
    ``offsets[j]:offsets[j+1]``) or "coupled" (dense rows, ``A`` of shape [m, n]).
    ``C`` is the penalty of the regularized form (kappa = 2/C); ``inf`` means
    the unregularized problem.
    """

    kind: str
    y: np.ndarray
    A: np.ndarray
    b: np.ndarray
    lo: float = LO
    hi: float = HI
    C: float = math.inf
    offsets: np.ndarray | None = None
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.y.shape[0])

    @property
    def m(self) -> int:
        return int(self.b.shape[0])

    @property
    def dtype(self):
        return self.y.dtype

    def dense_rows(self) -> np.ndarray:
        """A as an [m, n] float64 matrix (block-diagonal rows for 'independent')."""
        if self.kind != "independent":
            a = np.asarray(self.A, dtype=np.float64)
            return a.reshape(self.m, self.n)
        rows = np.zeros((self.m, self.n))
        for j in range(self.m):
            s, e = int(self.offsets[j]), int(self.offsets[j + 1])
            rows[j, s:e] = self.A[s:e]
        return rows


def _step_point(rng: np.random.Generator, n: int) -> np.ndarray:
    """y = x_prev - 0.1 g with x_prev ~ U(0,1), g ~ N(0,1): a gradient step from
    a feasible density field (Alg. 3 forms rho~ = rho_t - alpha grad f)."""
    x_prev = rng.uniform(0.0, 1.0, n)
    g = rng.standard_normal(n)
    return x_prev - 0.1 * g


def volume_2d(seed: int, nx: int = 64, ny: int = 32, vf: float = 0.5,
              dtype=np.float64) -> Problem:
    """Single linear volume constraint sum(x)/n <= vf on an nx x ny grid
    (Sec. 4.1.1, eq. (mincomp) with V_f).  64x32, float64 is the small case."""
    n = nx * ny
    rng = np.random.default_rng(seed)
    y = _step_point(rng, n).astype(dtype)
    a = np.full(n, 1.0 / n).astype(dtype)
    return Problem("single", y, a.reshape(1, n), np.array([vf]),
                   meta={"name": f"volume_{nx}x{ny}", "seed": seed})


def _planted_b(y: np.ndarray, a: np.ndarray, lam: float, lo: float, hi: float) -> float:
    """Right-hand side b = sum_i a_i clip(y_i - lam a_i) (exactly rounded sum),
    so that lam is the multiplier of the generated instance."""
    x = np.minimum(np.maximum(y - lam * a, lo), hi)
    return math.fsum((a * x).tolist())


def _lambda_for_free_fraction(y: np.ndarray, a: np.ndarray, frac: float,
                              lo: float, hi: float) -> float:
    """Recipe helper: the multiplier at which the fraction of elements with
    lo <= y - lam a <= hi is closest to ``frac`` (searching lam >= 0, a < 0)."""
    aa = np.abs(a)
    start = np.sort((lo - y) / aa)      # element enters [lo, hi] (a < 0 lifts z)
    end = np.sort((hi - y) / aa)        # element leaves through hi

    def free_frac(lam: float) -> float:
        return (np.searchsorted(start, lam, "right") - np.searchsorted(end, lam, "left")) / y.size

    lo_l, hi_l = 0.0, float(end[-1]) + 1.0
    for _ in range(200):
        mid = 0.5 * (lo_l + hi_l)
        if free_frac(mid) > frac:
            lo_l = mid
        else:
            hi_l = mid
    return 0.5 * (lo_l + hi_l)


def compliance_3d(seed: int, shape=(256, 128, 128), free_frac: float = 0.4,
                  dtype=np.float32, n: int | None = None) -> Problem:
    """Single linearized compliance constraint at scale (Sec. 4.1.2).

    a = dC/dx stand-in: -(|N(0,1)| + 0.01).  b is planted so that about
    ``free_frac`` of the elements are free at the solution.
    256x128x128 = 4,194,304 elements, float32 is the at-scale case."""
    if n is None:
        n = int(np.prod(shape))
    rng = np.random.default_rng(seed)
    y = _step_point(rng, n).astype(dtype)
    a = (-(np.abs(rng.standard_normal(n)) + 0.01)).astype(dtype)
    y64, a64 = y.astype(np.float64), a.astype(np.float64)
    lam = _lambda_for_free_fraction(y64, a64, free_frac, LO, HI)
    b = _planted_b(y64, a64, lam, LO, HI)
    return Problem("single", y, a.reshape(1, n), np.array([b]),
                   meta={"name": "compliance_%dx%dx%d" % tuple(shape) if n == int(np.prod(shape)) else f"compliance_n{n}",
                         "seed": seed, "planted_lambda": lam})


def multi_material(seed: int, fields: int = 4, n_per: int = 524288,
                   caps=(0.1, 0.1, 0.15, 0.15), dtype=np.float32) -> Problem:
    """Independent per-material volume constraints (Sec. 4.1.3): ``fields``
    contiguous fields of ``n_per`` elements, sum_{i in M_j} x_i / n_per <= cap_j.
    4 x 524,288 (a 1024x512 grid per field), float32 is the at-scale case."""
    n = fields * n_per
    rng = np.random.default_rng(seed)
    y = rng.uniform(-0.2, 1.2, n).astype(dtype)
    c = np.full(n, 1.0 / n_per).astype(dtype)
    offsets = np.arange(fields + 1, dtype=np.int64) * n_per
    caps = np.resize(np.asarray(caps, dtype=np.float64), fields)
    return Problem("independent", y, c, caps, offsets=offsets,
                   meta={"name": f"multimaterial_{fields}x{n_per}", "seed": seed})


def volume_com(seed: int, grid=(192, 96, 96), vf: float = 0.3, target=(0.25, 0.25),
               band=(0.02, 0.01), feasible: bool | None = None, C: float = C_DEFAULT,
               dtype=np.float32) -> Problem:
    """Coupled volume + centre-of-mass rows (Sec. 4.1.4), made linear.

    Domain [0,1] x [0,0.5] (x [0,0.5] in 3-D), element edge 1/nx, centroids at
    (i+1/2)/nx.  Rows: volume a = 1/n, b = vf; COM_x <= X_t + band_x and
    COM_x >= X_t - band_x, and the same in y, each multiplied through by
    sum(x) > 0 so that they are linear with b = 0.  m = 5, rank(A) = 3.
    ``feasible=False`` (default for odd seeds) moves the x-target to 0, which
    makes the box-constrained rows infeasible and exercises the regularized form.
    """
    nx, ny = grid[0], grid[1]
    nz = grid[2] if len(grid) > 2 else 1
    n = nx * ny * nz
    h = 1.0 / nx
    if feasible is None:
        feasible = (seed % 2 == 0)
    xt, yt = target
    if not feasible:
        xt = 0.0
    rng = np.random.default_rng(seed)
    y = _step_point(rng, n).astype(dtype)
    cx = (np.arange(nx) + 0.5) * h
    cy = (np.arange(ny) + 0.5) * h
    CX = np.repeat(cx, ny * nz)
    CY = np.tile(np.repeat(cy, nz), nx)
    bx, by = band
    rows = np.stack([
        np.full(n, 1.0 / n),
        (CX - xt - bx) / n,
        (xt - bx - CX) / n,
        (CY - yt - by) / n,
        (yt - by - CY) / n,
    ]).astype(dtype)
    b = np.array([vf, 0.0, 0.0, 0.0, 0.0])
    if not feasible:
        r = rows[1].astype(np.float64)
        xmin = np.where(r > 0, LO, HI)
        assert math.fsum((r * xmin).tolist()) > 0.0, "generator: COM row should be infeasible"
    name = "volcom_" + "x".join(str(g) for g in grid)
    return Problem("coupled", y, rows, b, C=C,
                   meta={"name": name, "seed": seed, "feasible": feasible})


def many_rows(seed: int, m: int = 64, grid=(256, 128, 128), active=None, eq_rows=(),
              C: float = C_DEFAULT, shift: float = 0.3, margin: float = 1e-3,
              dtype=np.float32) -> Problem:
    """m dense coupled rows with a planted multiplier: the large-m case of
    Alg. 2, where the Jacobian sums A D A^T of eq. (reg_jacobian) dominate a
    Newton pass (the remark in Sec. 4.2.1 that the Jacobian is built from the
    free variables only).

    Domain [0,1] x [0, ny/nx] x [0, nz/nx], element centroids as in
    ``volume_com``.  Rows: 0 the volume row 1/n; 1..ceil((m-1)/2) stand-ins
    for compliance sensitivities of separate load cases, -(|N(0,1)| + 0.01)
    times a smooth bump around a random load point plus 0.1, over n (they
    concentrate near their load, as dC/dx does); the rest moment rows,
    cos(pi kx X) cos(pi ky Y) cos(pi kz Z) / n with distinct random
    frequency triples in {0..3}^3 (sign-varying, like the centre-of-mass
    rows).

    Planting: lam*_j = s u_j, u_j ~ U(0.5, 1.5), on the rows in ``active``
    (default every fourth row, from row 0), s chosen so that the rms of
    A^T lam* is ``shift``; rows in ``eq_rows`` are equalities and take
    u_j of either sign.  With x* = clip(y - A^T lam*) (from the rounded
    arrays, in float64), b_j = a_j.x* - kappa lam*_j on active rows and
    a_j.x* + margin sigma_j on the others, so lam* satisfies the optimality
    conditions of Appendix A.2 and is the multiplier (unique for kappa > 0).
    The dot products are float64 BLAS sums (n is large here); the planted
    multiplier is exact for b up to their rounding."""
    nx, ny = grid[0], grid[1]
    nz = grid[2] if len(grid) > 2 else 1
    n = nx * ny * nz
    rng = np.random.default_rng(seed)
    y = _step_point(rng, n).astype(dtype)
    h = 1.0 / nx
    X = np.repeat((np.arange(nx) + 0.5) * h, ny * nz)
    Y = np.tile(np.repeat((np.arange(ny) + 0.5) * h, nz), nx)
    Z = np.tile((np.arange(nz) + 0.5) * h, nx * ny)
    ext = np.array([1.0, ny * h, nz * h])
    A = np.empty((m, n), dtype=dtype)
    A[0] = 1.0 / n
    ncomp = (m - 1 + 1) // 2
    # moment rows take distinct frequency triples (no two rows alike)
    triples = [(a, b_, c) for a in range(4) for b_ in range(4) for c in range(4) if (a, b_, c) != (0, 0, 0)]
    order = rng.permutation(len(triples))
    for j in range(1, m):
        if j <= ncomp:
            p = rng.uniform(0.0, 1.0, 3) * ext
            d2 = (X - p[0]) ** 2 + (Y - p[1]) ** 2 + (Z - p[2]) ** 2
            w = np.exp(-d2 / (2.0 * 0.15 ** 2)) + 0.1
            A[j] = (-(np.abs(rng.standard_normal(n)) + 0.01) * w / n).astype(dtype)
        else:
            kx, ky, kz = triples[order[j - ncomp - 1]]
            A[j] = (np.cos(np.pi * kx * X) * np.cos(np.pi * ky * Y / ext[1]) *
                    np.cos(np.pi * kz * Z / ext[2]) / n).astype(dtype)
    del X, Y, Z
    act = np.zeros(m, dtype=bool)
    if active is None:
        act[::4] = True
    else:
        act[list(active)] = True
    eq = np.zeros(m, dtype=bool)
    eq[list(eq_rows)] = True
    act |= eq
    u = rng.uniform(0.5, 1.5, m) * np.where(eq, rng.choice([-1.0, 1.0], m), 1.0)
    u = np.where(act, u, 0.0)
    y64 = y.astype(np.float64)
    dirv = np.zeros(n)
    for j in np.flatnonzero(act):
        dirv += u[j] * A[j].astype(np.float64)
    scale = shift / max(float(np.sqrt(np.mean(dirv * dirv))), 1e-300)
    lam = u * scale
    xs = np.minimum(np.maximum(y64 - scale * dirv, LO), HI)
    del dirv
    kappa = 0.0 if math.isinf(C) else 2.0 / C
    b = np.empty(m)
    sig = np.empty(m)
    for j in range(m):
        aj = A[j].astype(np.float64)
        ax = float(np.dot(aj, xs))
        sig[j] = float(np.sum(np.abs(aj))) * max(abs(LO), abs(HI))
        b[j] = ax - kappa * lam[j] if act[j] else ax + margin * sig[j]
    eq_mask = 0
    for j in np.flatnonzero(eq):
        eq_mask |= 1 << int(j)
    return Problem("coupled", y, A, b, C=C,
                   meta={"name": f"many_rows_m{m}_" + "x".join(str(g) for g in grid), "seed": seed,
                         "planted_lambda": lam, "active": act, "eq_mask": eq_mask})


@dataclass
class PgdState:
    """Caller-owned PGD state for one step of Alg. 3 (arrays in the stream dtype)."""
    rho: np.ndarray
    rho_prev: np.ndarray
    grad: np.ndarray
    grad_prev: np.ndarray
    d_prev: np.ndarray
    problem: Problem          # A = grad g(rho_t); y and b are formed by the step
    g: np.ndarray             # constraint values g_j(rho_t)
    G: np.ndarray             # bounds G_j
    t: int


def pgd_compliance_3d(seed: int, t: int = 60, shape=(256, 128, 128), n: int | None = None,
                      dtype=np.float32) -> PgdState:
    """One Alg. 3 step on the at-scale single-constraint case.

    rho_t = x_prev, grad f = g (the draws of the projection case),
    rho_{t-1} = rho_t - 0.01 N, grad f_{t-1} = g + 0.1 N, d_{t-1} = -grad f_{t-1}.
    The constraint is planted so that b = G - g + a.rho_t equals the planted
    right-hand side of ``compliance_3d`` for the same seed."""
    base = compliance_3d(seed, shape=shape, dtype=dtype, n=n)
    nn = base.n
    rng = np.random.default_rng(seed)
    x_prev = rng.uniform(0.0, 1.0, nn)
    g = rng.standard_normal(nn)
    rng2 = np.random.default_rng(seed + 1_000_003)
    rho = np.clip(x_prev, LO, HI).astype(dtype)
    grad = g.astype(dtype)
    rho_prev = (rho.astype(np.float64) - 0.01 * rng2.standard_normal(nn)).astype(dtype)
    grad_prev = (grad.astype(np.float64) + 0.1 * rng2.standard_normal(nn)).astype(dtype)
    d_prev = (-grad_prev.astype(np.float64)).astype(dtype)
    a64 = base.A.astype(np.float64).reshape(-1)
    arho = math.fsum((a64 * rho.astype(np.float64)).tolist())
    gval = np.array([arho])
    G = np.array([base.b[0]])
    prob = Problem("single", rho.copy(), base.A, np.array([np.nan]),
                   meta=dict(base.meta, name="pgd_" + base.meta["name"]))
    return PgdState(rho, rho_prev, grad, grad_prev, d_prev, prob, gval, G, t)


# --------------------------------------------------------------------------- serving

SERVE_KINDS = ("single", "independent", "coupled")


def serve_request(seed: int, n_target: int, kind: str, dtype=np.float32) -> Problem:
    """A request of the served stream at roughly ``n_target`` elements."""
    if kind == "single":
        return compliance_3d(seed, n=n_target, dtype=dtype)
    if kind == "independent":
        per = max(1, n_target // 4)
        return multi_material(seed, fields=4, n_per=per, dtype=dtype)
    if kind == "coupled":
        ny = max(2, int(round(math.sqrt(n_target / 2.0))))
        return volume_com(seed, grid=(2 * ny, ny), dtype=dtype)
    raise ValueError(kind)


def serve_stream(seed: int = 0, count: int = 4096, n_min: int = 4096, n_max: int = 2097152):
    """The served-batch stream: ``count`` requests, n log-uniform in [n_min, n_max],
    kind uniform over single / 4 independent / 5 coupled, one seed per request.
    Returns a list of (request_seed, kind, n_target); arrival times are drawn by
    the caller from an exponential distribution at its chosen rate."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        kind = SERVE_KINDS[int(rng.integers(0, 3))]
        s = int(rng.integers(0, 2**31 - 1))
        out.append((s, kind, n))
    return out
