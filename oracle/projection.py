"""Plain float64 statement of the projection subproblem of PGD-TO.

TEST INFRASTRUCTURE ONLY (see the package docstring): imported by tests/,
__graft_entry__.smoke() and bench.py's CPU-baseline leg, never by the product.

Notation.  The paper writes the multiplier as y <= 0 with delta = clip(sum_j y_j
grad g_j, l - rho~, u - rho~) (Theorem 1).  Here lam = -y >= 0, the point to
project is ``y`` (the paper's rho~), and x = rho~ + delta, so that

    x(lam) = clip(y - A^T lam, lo, hi)                       (Theorems 1 and 2)
    h_j(lam) = a_j . x(lam) - b_j - kappa lam_j              (Appendix A.2, eq. h)

with b_j = G_j - g_j(rho_t) + a_j . rho_t, so that the paper's G-hat is
b_j - a_j . rho~, and kappa = 2/C as printed in eq. (h) and eq. (reg_jacobian)
(kappa = 0 is the unregularized problem, eq. (linearized)).

The solution is the unique x = x(lam*) where lam* >= 0, h(lam*) <= 0 and
lam*_j h_j(lam*) = 0 (the three conditions that close Appendix A.2).  Every
function below computes that object by a route that can be checked by eye.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass

import numpy as np

try:                                     # optional: L-BFGS-B for the coupled dual
    from scipy.optimize import minimize as _sp_minimize
except Exception:                        # pragma: no cover - scipy is in the image
    _sp_minimize = None


# ----------------------------------------------------------------- primitives

def fsum(v) -> float:
    """Correctly rounded sum of a float64 vector."""
    return math.fsum(np.asarray(v, dtype=np.float64).ravel().tolist())


def clip_map(y, A, lam, lo, hi):
    """x(lam) = clip(y - A^T lam, lo, hi) and z = y - A^T lam.

    Theorem 1 / eq. (delta_y): delta_i is sum_j y_j a_ji clipped to
    [l - rho~_i, u - rho~_i]; with lam = -y_paper this is the box clip of z."""
    y = np.asarray(y, dtype=np.float64)
    A = np.atleast_2d(np.asarray(A, dtype=np.float64))
    lam = np.asarray(lam, dtype=np.float64).reshape(-1)
    z = y.copy()
    for j in range(A.shape[0]):          # one row at a time, as in sum_j lam_j a_j
        if lam[j] != 0.0:
            z = z - lam[j] * A[j]
    return np.minimum(np.maximum(z, lo), hi), z


def h_map(y, A, b, lam, lo, hi, kappa):
    """h_j(lam) = a_j . x(lam) - b_j - kappa lam_j  (eq. (h), lam = -y_paper)."""
    A = np.atleast_2d(np.asarray(A, dtype=np.float64))
    lam = np.asarray(lam, dtype=np.float64).reshape(-1)
    x, _ = clip_map(y, A, lam, lo, hi)
    return np.array([fsum(A[j] * x) - b[j] - kappa * lam[j] for j in range(A.shape[0])])


def row_scale(A, lo, hi):
    """sigma_j = sum_i |a_ji| max(|lo|, |hi|): the size of a_j . x over the box,
    used to express constraint tolerances relative to each row."""
    A = np.atleast_2d(np.asarray(A, dtype=np.float64))
    return np.array([fsum(np.abs(A[j])) for j in range(A.shape[0])]) * max(abs(lo), abs(hi))


# ------------------------------------------------------------- one row (m = 1)

def exact_single(y, a, b, lo, hi, kappa=0.0, eq=False):
    """Exact multiplier of the one-row projection.

    eq=True: the row is an equality a.x = b (Sec. 3.2, the note on equality
    constraints: always active, multiplier of either sign).  When phi(0) < 0
    the row a.x >= b, i.e. (-a).x <= -b, is the active one: it is solved as
    such and its multiplier negated (x = clip(y - lam a) with lam < 0).

    Appendix A.1 (eq. Gamma): with one row, phi(lam) = sum_i a_i clip(y_i - lam
    a_i) - b - kappa lam is piecewise linear and nonincreasing in lam (the
    paper's Gamma sum is nondecreasing in y = -lam).  Its kinks are the
    breakpoints (y_i - lo)/a_i and (y_i - hi)/a_i.  The root is found the way
    the cited Pardalos-Kovoor method does: locate the two neighbouring
    breakpoints between which phi changes sign (binary search over the sorted
    breakpoints), then solve the linear piece between them exactly.

    Returns (lam, outcome) with outcome in {"inactive", "converged", "infeasible"}:
      * phi(0) <= 0: the row is inactive, lam = 0 (Alg. 1 first branch).
      * kappa = 0 and phi stays positive past the last breakpoint: no point of
        the box satisfies the row; lam = the last breakpoint, i.e. every element
        with a_i != 0 sits at the bound that minimizes a_i x_i (this is where
        Algorithm 1's bracket collapses, y_u -> y_l).
      * kappa > 0: past the last breakpoint phi is linear with slope -kappa, so
        the root is last + phi(last)/kappa; the outcome is "infeasible" when
        the saturated point still violates the row (positive slack).
      * On a zero-slope stretch (kappa = 0) the smallest root is returned,
        which is the point Algorithm 1's "else y_l = y_m" rule converges to.
    """
    y = np.asarray(y, dtype=np.float64)
    a = np.asarray(a, dtype=np.float64)

    def phi(lam, exact=False):
        x = np.minimum(np.maximum(y - lam * a, lo), hi)
        s = fsum(a * x) if exact else float(np.sum(a * x))
        return s - b - kappa * lam

    if eq:
        p0 = phi(0.0, exact=True)
        if p0 == 0.0:
            return 0.0, "converged"
        if p0 < 0.0:
            lam, out = exact_single(y, -a, -b, lo, hi, kappa)
            return -lam, out
    if phi(0.0, exact=True) <= 0.0:
        return 0.0, "inactive"
    nz = a != 0.0
    bp = np.concatenate([(y[nz] - lo) / a[nz], (y[nz] - hi) / a[nz]])
    bp = np.unique(bp[bp > 0.0])
    last = float(bp[-1]) if bp.size else 0.0
    phi_last = phi(last, exact=True)
    if phi_last > 0.0:
        # every element with a_i != 0 is saturated for lam >= last
        x_sat = np.where(a > 0, lo, np.where(a < 0, hi, 0.0))
        viol = fsum(a * x_sat) - b
        if kappa > 0.0:
            return last + phi_last / kappa, ("infeasible" if viol > 0.0 else "converged")
        return last, "infeasible"
    # binary search for adjacent breakpoints with phi(left) > 0 >= phi(right)
    i_lo, i_hi = -1, bp.size - 1            # i_lo = -1 stands for lam = 0
    while i_hi - i_lo > 1:
        mid = (i_lo + i_hi) // 2
        if phi(float(bp[mid])) > 0.0:
            i_lo = mid
        else:
            i_hi = mid
    left = 0.0 if i_lo < 0 else float(bp[i_lo])
    right = float(bp[i_hi])
    # on (left, right) no element changes state: phi is linear there, with
    # slope -(sum of a_i^2 over the free elements + kappa)
    probe = 0.5 * (left + right)
    zp = y - probe * a
    free = (zp >= lo) & (zp <= hi)
    slope = fsum(a[free] ** 2) + kappa
    pl = phi(left, exact=True)
    if pl <= 0.0:                            # rounding put the root at `left`
        return left, "converged"
    lam = left + pl / slope
    return min(max(lam, left), right), "converged"


# ------------------------------------------------------------ coupled rows

def _dual_value_grad(lam, y, A, b, lo, hi, kappa):
    """q(lam) = 1/2 ||x(lam) - y||^2 + lam.(A x(lam) - b) - kappa/2 ||lam||^2 and
    its gradient h(lam): the Lagrangian dual of the regularized problem
    (eq. regularized), whose maximizer over lam >= 0 is lam*."""
    x, _ = clip_map(y, A, lam, lo, hi)
    Ax = A @ x
    q = 0.5 * float(np.dot(x - y, x - y)) + float(np.dot(lam, Ax - b)) - 0.5 * kappa * float(np.dot(lam, lam))
    return q, Ax - b - kappa * lam


def _polish(lam, y, A, b, lo, hi, kappa, max_iter=200, eq=None):
    """Fix the element pattern (lower / free / upper) and the active rows at the
    current lam and solve the resulting linear system for lam exactly:

        (A_SF A_SF^T + kappa I) lam_S = A_SF y_F + lo A_SL 1 + hi A_SU 1 - b_S

    which is h_S(lam) = 0 written out for that pattern (eq. h with x from
    eq. delta_y_robust).  Repeat until the pattern no longer changes.
    Equality rows (eq) are always in S and keep multipliers of either sign."""
    m = A.shape[0]
    eq = np.zeros(m, dtype=bool) if eq is None else np.asarray(eq, dtype=bool)
    lam = np.asarray(lam, dtype=np.float64)
    lam = np.where(eq, lam, np.maximum(lam, 0.0))
    seen = set()
    for _ in range(max_iter):
        x, z = clip_map(y, A, lam, lo, hi)
        F = (z >= lo) & (z <= hi)
        L = z < lo
        U = z > hi
        h = np.array([fsum(A[j] * x) - b[j] - kappa * lam[j] for j in range(m)])
        S = eq | (lam > 0.0) | (h > 0.0)
        key = (S.tobytes(), np.packbits(F).tobytes(), np.packbits(L).tobytes())
        new = np.zeros(m)
        if S.any():
            AS = A[S]
            AF = AS[:, F]
            M = AF @ AF.T + kappa * np.eye(int(S.sum()))
            rhs = AF @ y[F] + lo * AS[:, L].sum(axis=1) + hi * AS[:, U].sum(axis=1) - b[S]
            try:
                sol = np.linalg.solve(M, rhs)
            except np.linalg.LinAlgError:
                sol = np.linalg.lstsq(M, rhs, rcond=None)[0]
            for _r in range(2):      # refinement with an exactly summed residual
                full = np.zeros(m)
                full[S] = sol
                xr, _ = clip_map(y, A, full, lo, hi)
                res = np.array([fsum(A[j] * xr) - b[j] - kappa * full[j] for j in np.flatnonzero(S)])
                # on a fixed pattern, h_S(lam) = rhs - M lam_S
                zr = y - A.T @ full
                if not (np.array_equal((zr >= lo) & (zr <= hi), F)):
                    break
                try:
                    sol = sol + np.linalg.solve(M, res)
                except np.linalg.LinAlgError:
                    break
            new[S] = sol
        new = np.where(eq, new, np.maximum(new, 0.0))
        if np.array_equal(new, lam) or key in seen:
            lam = new
            break
        seen.add(key)
        lam = new
    return lam


def coupled(y, A, b, lo, hi, kappa, lam0=None, eq=None):
    """Multiplier of the regularized multi-row projection (Appendix A.2).

    1. Maximize the concave dual q over lam >= 0 (L-BFGS-B on -q with Jacobi
       scaling; gradient h), which is a plain way to approach lam*.
    2. Polish: solve the fixed-pattern linear system exactly (``_polish``).
    Correctness is established independently by ``kkt_certificate`` (the
    solution is unique when kappa > 0: Appendix A.2, eq. reg_jacobian).
    Equality rows (eq, Sec. 3.2): the dual variable is free in sign."""
    y = np.asarray(y, dtype=np.float64)
    A = np.atleast_2d(np.asarray(A, dtype=np.float64))
    b = np.asarray(b, dtype=np.float64)
    m = A.shape[0]
    eq = np.zeros(m, dtype=bool) if eq is None else np.asarray(eq, dtype=bool)
    h0 = h_map(y, A, b, np.zeros(m), lo, hi, kappa)
    if np.all(h0[~eq] <= 0.0) and np.all(h0[eq] == 0.0):
        return np.zeros(m)
    d = np.array([float(np.dot(A[j], A[j])) for j in range(m)]) + kappa
    d[d == 0.0] = 1.0
    start = np.zeros(m) if lam0 is None else np.asarray(lam0, float)
    start = np.where(eq, start, np.maximum(start, 0.0))
    lam = start
    if _sp_minimize is not None:
        def f(mu):
            q, g = _dual_value_grad(mu / d, y, A, b, lo, hi, kappa)
            return -q, -g / d
        res = _sp_minimize(f, start * d, jac=True, method="L-BFGS-B",
                           bounds=[(None, None) if e else (0.0, None) for e in eq],
                           options={"maxiter": 5000, "ftol": 1e-16, "gtol": 1e-14, "maxcor": 20})
        lam = res.x / d
        lam = np.where(eq, lam, np.maximum(lam, 0.0))
    return _polish(lam, y, A, b, lo, hi, kappa, eq=eq)


# ------------------------------------------------------------ KKT certificate

def kkt_certificate(y, A, b, lo, hi, kappa, lam, x=None, eq=None):
    """Scaled residuals of the KKT system of the regularized problem
    (eqs. rkkt1-rkkt11, reduced as in Appendix A.2 to conditions on lam):

      map     max_i |x_i - clip(y - A^T lam)_i|
      dual    -min_j lam_j                       (lam >= 0)
      primal  max_j max(h_j, 0) / sigma_j        (h <= 0)
      compl   max_j |lam_j h_j| / (sigma_j max(1, lam_j))
    Equality rows (eq): lam_j of either sign, primal |h_j| / sigma_j, no
    complementarity term.
    """
    A = np.atleast_2d(np.asarray(A, dtype=np.float64))
    lam = np.asarray(lam, dtype=np.float64).reshape(-1)
    eq = np.zeros(lam.size, dtype=bool) if eq is None else np.asarray(eq, dtype=bool)
    xl, _ = clip_map(y, A, lam, lo, hi)
    sig = row_scale(A, lo, hi)
    sig[sig == 0.0] = 1.0
    h = h_map(y, A, b, lam, lo, hi, kappa)
    ine = ~eq
    out = {
        "map": 0.0 if x is None else float(np.max(np.abs(np.asarray(x, float) - xl), initial=0.0)),
        "dual": float(max(0.0, -np.min(lam[ine], initial=0.0))),
        "primal": float(np.max(np.where(eq, np.abs(h), np.maximum(h, 0.0)) / sig)),
        "compl": float(np.max(np.abs(lam[ine] * h[ine]) / (sig[ine] * np.maximum(1.0, lam[ine])), initial=0.0)),
    }
    out["max"] = max(out.values())
    return out


# ------------------------------------------------------------ brute force

def brute_force(y, A, b, lo, hi, kappa, tol=1e-9, eq=None):
    """Enumerate every element state in {lower, upper, free}^n and every set S
    of rows held at equality, solve the KKT equations of that combination, and
    keep the combinations that satisfy all sign conditions (Appendix A: the
    case analysis behind eq. delta_y plus conditions 1-3 on y).  Returns the
    list of surviving x vectors (uniqueness says they all coincide).
    Equality rows (eq) belong to every S and may take multipliers of either
    sign.  For n <= 9 and m <= 3 only."""
    y = np.asarray(y, dtype=np.float64)
    A = np.atleast_2d(np.asarray(A, dtype=np.float64))
    b = np.asarray(b, dtype=np.float64)
    m, n = A.shape
    eq = np.zeros(m, dtype=bool) if eq is None else np.asarray(eq, dtype=bool)
    states = np.array(list(itertools.product((0, 1, 2), repeat=n)))   # 0 L, 1 U, 2 F
    survivors = []
    for r in range(m + 1):
        for S in itertools.combinations(range(m), r):
            S = list(S)
            if any(eq[j] and j not in S for j in range(m)):
                continue
            for st in states:
                F = st == 2
                xf = np.where(st == 0, lo, np.where(st == 1, hi, 0.0))
                lam = np.zeros(m)
                if S:
                    AS = A[S]
                    M = AS[:, F] @ AS[:, F].T + kappa * np.eye(len(S))
                    rhs = AS[:, F] @ y[F] + AS[:, ~F] @ xf[~F] - b[S]
                    if abs(np.linalg.det(M)) < 1e-300:
                        continue
                    lam[S] = np.linalg.solve(M, rhs)
                z = y - A.T @ lam
                x = np.where(F, z, xf)
                if np.any(lam[~eq] < -tol):
                    continue
                if np.any(z[st == 0] > lo + tol) or np.any(z[st == 1] < hi - tol):
                    continue
                if np.any(z[F] < lo - tol) or np.any(z[F] > hi + tol):
                    continue
                h = A @ x - b - kappa * lam
                notS = [j for j in range(m) if j not in S]
                if notS and np.any(h[notS] > tol):
                    continue
                if S and np.any(np.abs(h[S]) > tol):
                    continue
                survivors.append(x)
    return survivors


# ------------------------------------------------------------ dispatcher

@dataclass
class OracleResult:
    x: np.ndarray          # projected point, float64
    z: np.ndarray          # y - A^T lam (pre-clip), float64
    lam: np.ndarray        # multipliers (lam = -y_paper >= 0)
    outcome: list          # per row / block
    resid: np.ndarray      # a_j . x - b_j
    slack: np.ndarray      # kappa lam_j (eq. s_y_robust: s = -2 y / C)
    n_free: int            # elements with lo <= z <= hi
    kappa: float


def largest_breakpoint(y, a, lo, hi):
    """Largest multiplier at which an element of one row reaches the bound it
    is driven to: (y_i - lo)/a_i for a_i > 0, (y_i - hi)/a_i for a_i < 0,
    elements with a_i = 0 left out (Appendix A.1; the end of Algorithm 1's
    bracket, -y_l in the paper's sign).  -inf for a row without coefficients."""
    y = np.asarray(y, dtype=np.float64)
    a = np.asarray(a, dtype=np.float64)
    best = -math.inf
    for yi, ai in zip(y, a):
        if ai > 0.0:
            best = max(best, (yi - lo) / ai)
        elif ai < 0.0:
            best = max(best, (yi - hi) / ai)
    return best


def auto_C(kind, y, A, lo, hi, tau, offsets=None):
    """The penalty of Appendix A.2 that bounds the constraint violation by
    tau: C = 2 bp / tau with bp the largest breakpoint over all rows (the
    paper writes the smallest breakpoint in its sign, y <= 0, whose magnitude
    this is), so kappa = 2/C = tau / bp.  inf (kappa = 0) when no breakpoint
    is positive."""
    y = np.asarray(y, dtype=np.float64)
    if kind == "independent":
        c = np.asarray(A, dtype=np.float64).reshape(-1)
        rows = [(y[int(offsets[j]):int(offsets[j + 1])], c[int(offsets[j]):int(offsets[j + 1])])
                for j in range(len(offsets) - 1)]
    else:
        Ad = np.atleast_2d(np.asarray(A, dtype=np.float64))
        rows = [(y, Ad[j]) for j in range(Ad.shape[0])]
    bp = max(largest_breakpoint(yy, aa, lo, hi) for yy, aa in rows)
    if not (bp > 0.0) or not math.isfinite(bp):
        return math.inf
    return 2.0 * bp / tau


def project(kind, y, A, b, lo, hi, C=math.inf, offsets=None, eq=None):
    """Projection of y onto {lo <= x <= hi, A x <= b} in the regularized form
    with kappa = 2/C (kappa = 0 when C is infinite).  eq (optional, one flag
    per row or block): rows held at equality, a_j.x = b_j (Sec. 3.2).

    kind "single": one dense row (Algorithm 1's problem).
    kind "independent": disjoint blocks, A[i] is the coefficient of element i in
        the row of the block that owns it (Sec. 3.2.2: separate 1-row problems).
    kind "coupled": dense rows (Algorithm 2's problem)."""
    y = np.asarray(y, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    kappa = 0.0 if math.isinf(C) else 2.0 / C
    n = y.size
    m_rows = b.size
    eq = np.zeros(m_rows, dtype=bool) if eq is None else np.asarray(eq, dtype=bool).reshape(-1)
    if kind == "independent":
        c = np.asarray(A, dtype=np.float64).reshape(-1)
        m = b.size
        lam = np.zeros(m)
        outcome = []
        x = np.empty(n)
        z = np.empty(n)
        for j in range(m):
            s, e = int(offsets[j]), int(offsets[j + 1])
            lj, oj = exact_single(y[s:e], c[s:e], b[j], lo, hi, kappa, eq=bool(eq[j]))
            lam[j] = lj
            outcome.append(oj)
            z[s:e] = y[s:e] - lj * c[s:e]
        x = np.minimum(np.maximum(z, lo), hi)
        resid = np.array([fsum(c[int(offsets[j]):int(offsets[j + 1])] * x[int(offsets[j]):int(offsets[j + 1])]) - b[j]
                          for j in range(m)])
    else:
        Ad = np.atleast_2d(np.asarray(A, dtype=np.float64))
        m = Ad.shape[0]
        if kind == "single":
            lj, oj = exact_single(y, Ad[0], b[0], lo, hi, kappa, eq=bool(eq[0]))
            lam = np.array([lj])
            outcome = [oj]
        elif kind == "coupled":
            lam = coupled(y, Ad, b, lo, hi, kappa, eq=eq)
            outcome = ["inactive" if np.all(lam == 0.0) else "converged"]
        else:
            raise ValueError(kind)
        x, z = clip_map(y, Ad, lam, lo, hi)
        resid = np.array([fsum(Ad[j] * x) - b[j] for j in range(m)])
    n_free = int(np.count_nonzero((z >= lo) & (z <= hi)))
    return OracleResult(x, z, lam, outcome, resid, kappa * lam, n_free, kappa)


def kappa_path(kind, y, A, b, lo, hi, C_values, offsets=None, eq=None, tau=0.0):
    """The regularized projection along a list of penalties (Appendix A.2,
    the remark that closes the choice of C: for an infeasible subproblem, C
    trades the violation of the constraints against the distance the
    projection moves the point).  Every point is its own solve: the
    projection is unique for each kappa > 0, so no continuation is needed to
    define it.  A negative C asks for the automatic penalty with tau = -C.

    Per point: kappa, the multipliers, the slack kappa lam_j, the violation
    max(0, a_j.x - b_j) of every row (|a_j.x - b_j| for an equality row), its
    largest entry and 2-norm, the distance ||x - y||_2, and the largest
    violation over tau when tau > 0."""
    y = np.asarray(y, dtype=np.float64)
    m = np.asarray(b, dtype=np.float64).size
    eqa = np.zeros(m, dtype=bool) if eq is None else np.asarray(eq, dtype=bool).reshape(-1)
    pts = []
    for Cv in C_values:
        C_eff = auto_C(kind, y, A, lo, hi, -Cv, offsets) if Cv < 0 else Cv
        r = project(kind, y, A, b, lo, hi, C_eff, offsets, eq=eq)
        viol = np.where(eqa, np.abs(r.resid), np.maximum(r.resid, 0.0))
        dist = math.sqrt(fsum((r.x - y) ** 2))
        vmax = float(np.max(viol)) if viol.size else 0.0
        pts.append({"C": Cv, "kappa": r.kappa, "lam": r.lam.copy(), "slack": r.slack.copy(), "violation": viol,
                    "max_violation": vmax, "violation_norm": math.sqrt(fsum(viol ** 2)), "dist": dist,
                    "violation_over_tau": vmax / tau if tau > 0 else 0.0, "result": r})
    return pts
