"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: hand
derivations from Theorems 1/2 (golden fixtures), closed forms, brute-force
enumeration of the KKT case analysis (Appendix A), invariances stated in the
paper (independent blocks, regularization limit, uniqueness) and the paper's
literal Algorithm 1.  A test at the end plants mistakes in the oracle and
checks that these pins catch them.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import projection as P
from oracle import literal
from paper_2511_13905_amd import inputs as I

GOLD = os.path.join(os.path.dirname(__file__), "golden", "hand_worked.json")


def _C(v):
    return math.inf if v == "inf" else float(v)


@pytest.mark.parametrize("case", json.load(open(GOLD))["cases"], ids=lambda c: c["name"])
def test_hand_worked_cases(case):
    """Golden fixtures derived by hand from Theorems 1 and 2."""
    y = np.array(case["y"])
    A = np.array(case["A"])
    b = np.array(case["b"])
    r = oracle.project(case["kind"], y, A, b, case["lo"], case["hi"], _C(case["C"]))
    np.testing.assert_allclose(r.x, case["x"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(r.lam, case["lam"], rtol=1e-12, atol=1e-12)
    assert list((r.z >= case["lo"]) & (r.z <= case["hi"])) == case["free"]


@pytest.mark.parametrize("kappa", [0.0, 2e-12, 0.5])
def test_closed_form_all_free_uniform_row(kappa):
    """a = 1/n, every element free: lam = (mean(y) - b) / (1/n + kappa), x = y - lam/n."""
    rng = np.random.default_rng(7)
    n = 1000
    y = rng.uniform(0.4, 0.6, n)
    a = np.full(n, 1.0 / n)
    b = float(np.mean(y)) - 0.05
    C = math.inf if kappa == 0 else 2.0 / kappa
    r = oracle.project("single", y, a.reshape(1, n), [b], 0.0, 1.0, C)
    lam = (P.fsum(y) / n - b) / (1.0 / n + kappa)
    assert r.lam[0] == pytest.approx(lam, rel=1e-12)
    np.testing.assert_allclose(r.x, y - lam / n, rtol=0, atol=1e-13)
    assert r.n_free == n


def test_closed_form_infeasible_single_row_regularized():
    """One infeasible row, kappa > 0: x is the saturated point, lam = (a.x_sat - b)/kappa."""
    rng = np.random.default_rng(11)
    n = 500
    y = rng.uniform(-0.5, 1.5, n)
    a = rng.uniform(0.1, 1.0, n)
    lo, hi = 0.1, 1.0
    x_sat = np.full(n, lo)
    b = P.fsum(a * x_sat) - 3.0          # unreachable even at the lower bound
    kappa = 1e-3
    lam, outcome = P.exact_single(y, a, b, lo, hi, kappa)
    assert outcome == "infeasible"
    assert lam == pytest.approx((P.fsum(a * x_sat) - b) / kappa, rel=1e-12)
    x, _ = P.clip_map(y, a.reshape(1, n), [lam], lo, hi)
    np.testing.assert_array_equal(x, x_sat)


def test_infeasible_unregularized_is_saturated_point():
    """kappa = 0 and no box point satisfies the row: x = (a > 0 ? lo : hi) for a != 0,
    clip(y) for a = 0 (where Alg. 1's bracket collapses)."""
    rng = np.random.default_rng(12)
    n = 300
    y = rng.uniform(-0.5, 1.5, n)
    a = rng.standard_normal(n)
    a[::17] = 0.0
    lo, hi = 0.0, 1.0
    x_min = np.where(a > 0, lo, np.where(a < 0, hi, np.clip(y, lo, hi)))
    b = P.fsum(a * x_min) - 1.0
    r = oracle.project("single", y, a.reshape(1, n), [b], lo, hi)
    assert r.outcome == ["infeasible"]
    np.testing.assert_array_equal(r.x, x_min)


def test_inactive_is_bit_exact_clip():
    """If delta(0) is feasible the answer is y* = 0 (Alg. 1, first branch): x = clip(y) exactly."""
    p = I.volume_2d(0)
    r = oracle.project(p.kind, p.y, p.A, p.b, p.lo, p.hi)
    assert r.outcome == ["inactive"]
    np.testing.assert_array_equal(r.x, np.clip(p.y, p.lo, p.hi))


def _random_case(rng, n, m, kind):
    y = rng.uniform(-0.6, 1.6, n)
    A = rng.standard_normal((m, n))
    if kind == "infeasible":
        xmin = np.where(A[0] > 0, 0.0, 1.0)
        b = A @ np.clip(y, 0, 1) - 0.5
        b[0] = float(A[0] @ xmin) - 0.2
    else:
        # feasible by construction: a box point x0 satisfies every row
        if kind == "duplicate" and m >= 2:
            A[1] = A[0]
        x0 = rng.uniform(0.0, 1.0, n)
        b = A @ x0 + rng.uniform(0.0, 0.3, m)
        if kind == "duplicate" and m >= 2:
            b[1] = b[0]
    return y, A, b


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("m", [1, 2, 3])
@pytest.mark.parametrize("kappa", [0.0, 2e-12, 1.0])
@pytest.mark.parametrize("kind", ["random", "infeasible", "duplicate"])
def test_brute_force_agrees(seed, m, kappa, kind):
    """Enumerating all element states and active row sets (Appendix A case
    analysis) leaves exactly one x (uniqueness, Sec. 3.2.3), equal to the oracle's."""
    if kind == "infeasible" and kappa == 0.0:
        pytest.skip("no KKT point exists without regularization")
    if kind == "infeasible" and kappa < 1e-6:
        pytest.skip("lam ~ violation/kappa ~ 1e11: the enumerated solves cancel catastrophically")
    if kind == "duplicate" and m < 2:
        pytest.skip("needs two rows")
    rng = np.random.default_rng(1000 * seed + 10 * m + int(kappa > 0) + (5 if kappa == 1.0 else 0))
    n = 6 if m < 3 else 5
    y, A, b = _random_case(rng, n, m, kind)
    C = math.inf if kappa == 0 else 2.0 / kappa
    r = oracle.project("coupled" if m > 1 else "single", y, A, b, 0.0, 1.0, C)
    sv = P.brute_force(y, A, b, 0.0, 1.0, kappa)
    assert len(sv) >= 1
    for s in sv:
        np.testing.assert_allclose(s, sv[0], atol=1e-8)
    np.testing.assert_allclose(r.x, sv[0], atol=1e-8)


def test_alg1_literal_agrees_with_exact():
    """The paper's Algorithm 1 (bisection, tol_B) lands within tol_B of the exact root."""
    for seed in range(12):
        p = I.volume_2d(seed, vf=0.4)
        lam, out = P.exact_single(p.y, p.A[0], p.b[0], p.lo, p.hi)
        y_star, it = literal.alg1_bisection(p.y, p.A[0], p.b[0], p.lo, p.hi, tol_b=1e-8)
        assert abs(-y_star - lam) <= 1e-8 * max(1.0, lam) + 1e-12
    p = I.compliance_3d(3, n=20000)
    lam, _ = P.exact_single(p.y.astype(float), p.A[0].astype(float), p.b[0], p.lo, p.hi)
    y_star, _ = literal.alg1_bisection(p.y.astype(float), p.A[0].astype(float), p.b[0], p.lo, p.hi, tol_b=1e-10)
    assert abs(-y_star - lam) <= 1e-9


def test_coupled_with_one_row_equals_single():
    """Algorithm 2 with m = 1 solves the same problem as the 1-row search (kappa kept)."""
    rng = np.random.default_rng(5)
    n = 2000
    y = rng.uniform(-0.3, 1.3, n)
    a = rng.standard_normal(n)
    b = float(a @ np.clip(y, 0, 1)) - 4.0
    for kappa in (0.0, 1e-6, 1.0):
        lam_s, _ = P.exact_single(y, a, b, 0.0, 1.0, kappa)
        lam_c = P.coupled(y, a.reshape(1, n), [b], 0.0, 1.0, kappa)
        assert lam_c[0] == pytest.approx(lam_s, rel=1e-10)


def test_planted_duals_recovered():
    """Pick lam* >= 0, set b so that lam* satisfies the optimality conditions
    (active rows: h_j(lam*) = 0; inactive: h_j < 0) and recover it."""
    rng = np.random.default_rng(21)
    n, m = 5000, 4
    y = rng.uniform(-0.2, 1.2, n)
    A = rng.standard_normal((m, n)) / n
    lam_star = np.array([3.0, 0.0, 7.5, 0.0]) * n
    kappa = 2e-12
    x, _ = P.clip_map(y, A, lam_star, 0.0, 1.0)
    b = np.array([P.fsum(A[j] * x) for j in range(m)]) - kappa * lam_star
    b[1] += 0.05
    b[3] += 0.01
    r = oracle.project("coupled", y, A, b, 0.0, 1.0, 2.0 / kappa)
    np.testing.assert_allclose(r.lam, lam_star, rtol=1e-9, atol=1e-6)
    np.testing.assert_allclose(r.x, x, atol=1e-12)


def test_independent_blocks_equal_separate_solves():
    """Disjoint index sets decouple into separate 1-row problems (Sec. 3.2.2)."""
    p = I.multi_material(2, fields=4, n_per=3000)
    r = oracle.project(p.kind, p.y, p.A, p.b, p.lo, p.hi, offsets=p.offsets)
    for j in range(4):
        s, e = p.offsets[j], p.offsets[j + 1]
        rj = oracle.project("single", p.y[s:e], p.A[s:e].reshape(1, -1), p.b[j:j + 1], p.lo, p.hi)
        np.testing.assert_array_equal(r.x[s:e], rj.x)
        assert r.lam[j] == rj.lam[0]
    # and the dense block-diagonal form solved as coupled (kappa = 0) gives the same x
    rc = oracle.project("coupled", p.y, p.dense_rows(), p.b, p.lo, p.hi, math.inf)
    np.testing.assert_allclose(rc.x, r.x, atol=1e-10)


def test_row_scaling_invariance():
    """a_j -> c a_j, b_j -> c b_j leaves x unchanged at kappa = 0 and maps lam_j -> lam_j / c."""
    p = I.compliance_3d(4, n=30000, dtype=np.float64)
    r1 = oracle.project("single", p.y, p.A, p.b, p.lo, p.hi)
    c = 8.0
    r2 = oracle.project("single", p.y, c * p.A, c * p.b, p.lo, p.hi)
    np.testing.assert_allclose(r2.x, r1.x, atol=1e-13)
    assert r2.lam[0] == pytest.approx(r1.lam[0] / c, rel=1e-12)


def test_duplicate_rows_split_the_multiplier():
    """Two identical rows at kappa > 0 carry equal multipliers whose sum solves
    the single row with kappa/2 (regularization makes lam unique, eq. reg_jacobian;
    without it only the sum is fixed, eq. unreg_jacobian)."""
    rng = np.random.default_rng(9)
    n = 3000
    y = rng.uniform(-0.2, 1.2, n)
    a = rng.standard_normal(n) / n
    b = float(a @ np.clip(y, 0, 1)) - 1e-3
    kappa = 1e-6
    lam2 = P.coupled(y, np.stack([a, a]), [b, b], 0.0, 1.0, kappa)
    lam1, _ = P.exact_single(y, a, b, 0.0, 1.0, kappa / 2)
    assert lam2[0] == pytest.approx(lam2[1], rel=1e-8)
    assert lam2.sum() == pytest.approx(lam1, rel=1e-8)


def test_permutation_equivariance():
    p = I.volume_com(0, grid=(24, 12, 12))
    perm = np.random.default_rng(3).permutation(p.n)
    r1 = oracle.project(p.kind, p.y, p.A, p.b, p.lo, p.hi, p.C)
    r2 = oracle.project(p.kind, p.y[perm], p.A[:, perm], p.b, p.lo, p.hi, p.C)
    np.testing.assert_allclose(r2.x, r1.x[perm], atol=1e-12)


def test_regularization_limit():
    """C -> infinity recovers the unregularized projection (Sec. 3.2.3)."""
    rng = np.random.default_rng(14)
    n = 4000
    y = rng.uniform(-0.2, 1.2, n)
    A = rng.standard_normal((2, n)) / n
    b = A @ np.clip(y, 0, 1) - np.array([2e-4, 1e-4])
    r0 = oracle.project("coupled", y, A, b, 0.0, 1.0, math.inf)
    errs = []
    for C in (1e6, 1e9, 1e12):
        r = oracle.project("coupled", y, A, b, 0.0, 1.0, C)
        errs.append(float(np.max(np.abs(r.x - r0.x))))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-9


def test_auto_C_hand_example():
    """Appendix A.2's penalty C = 2 bp / tau on breakpoints worked by hand:
    y = (0.5, 0.2), a = (1, -2), box [0, 1]: element 1 reaches 0 at
    lam = 0.5/1, element 2 reaches 1 at lam = (0.2 - 1)/(-2) = 0.4; the
    largest is 0.5, so C = 2 * 0.5 / 1e-3 = 1000."""
    assert P.largest_breakpoint([0.5, 0.2], [1.0, -2.0], 0.0, 1.0) == 0.5
    assert oracle.auto_C("single", [0.5, 0.2], [[1.0, -2.0]], 0.0, 1.0, 1e-3) == 1000.0
    # two blocks: the largest over blocks (block 2: (0.9 - 0)/0.5 = 1.8)
    assert oracle.auto_C("independent", [0.5, 0.2, 0.9], [1.0, -2.0, 0.5], 0.0, 1.0, 1e-3,
                         offsets=[0, 2, 3]) == pytest.approx(2 * 1.8 / 1e-3, rel=1e-15)
    # coupled rows: the largest over rows
    assert oracle.auto_C("coupled", [0.5, 0.2], [[1.0, -2.0], [0.25, 0.0]], 0.0, 1.0, 1e-3) == 4000.0
    # no positive breakpoint (every element already at the bound it moves to): kappa = 0
    assert oracle.auto_C("single", [0.0, 1.0], [[1.0, -1.0]], 0.0, 1.0, 1e-3) == math.inf


@pytest.mark.parametrize("seed", range(4))
def test_auto_C_bounds_violation(seed):
    """With C = 2 bp / tau the regularized optimum violates a feasible row by
    at most tau (the bound stated with the penalty in Appendix A.2): the
    multiplier stays below bp, and the violation is kappa lam."""
    rng = np.random.default_rng(40 + seed)
    n = 3000
    y = rng.uniform(-0.2, 1.2, n)
    a = -(np.abs(rng.standard_normal(n)) + 0.01)
    lam0 = rng.uniform(0.2, 0.8)
    b = float(a @ np.clip(y - lam0 * a, 0.0, 1.0))        # planted, feasible
    tau = 10.0 ** rng.uniform(-6, -2) * abs(b)
    C = oracle.auto_C("single", y, a.reshape(1, -1), 0.0, 1.0, tau)
    r = oracle.project("single", y, a.reshape(1, -1), [b], 0.0, 1.0, C)
    viol = r.resid[0]
    assert 0.0 <= viol <= tau * (1 + 1e-9), (viol, tau)
    assert r.slack[0] == pytest.approx(viol, rel=1e-6, abs=1e-12 * abs(b))
    assert r.lam[0] <= P.largest_breakpoint(y, a, 0.0, 1.0)


@pytest.mark.parametrize("kappa", [0.0, 0.5])
def test_equality_row_closed_form(kappa):
    """An equality row a.x = b (Sec. 3.2: always active, multiplier of either
    sign) on a point that stays inside the box: x = y - lam a with
    a.(y - lam a) - b - kappa lam = 0, so lam = (a.y - b) / (a.a + kappa),
    negative when b lies above a.y."""
    n = 50
    y = 0.3 + 0.4 * np.arange(n) / n
    a = np.full(n, 1.0 / n)
    for shift in (+0.02, -0.02):                 # b above a.y (lam < 0), below (lam > 0)
        b = float(a @ y) + shift
        lam_cf = (float(a @ y) - b) / (float(a @ a) + kappa)
        lam, out = P.exact_single(y, a, b, 0.0, 1.0, kappa, eq=True)
        assert out == "converged"
        assert lam == pytest.approx(lam_cf, rel=1e-12)
        assert np.sign(lam) == -np.sign(shift)
        C = math.inf if kappa == 0.0 else 2.0 / kappa
        r = oracle.project("single", y, a.reshape(1, -1), [b], 0.0, 1.0, C, eq=[True])
        assert r.lam[0] == pytest.approx(lam_cf, rel=1e-12)
        rc = oracle.project("coupled", y, a.reshape(1, -1), [b], 0.0, 1.0, C, eq=[True])
        assert rc.lam[0] == pytest.approx(lam_cf, rel=1e-9)
    # an inequality row with b above a.y is inactive instead
    r = oracle.project("single", y, a.reshape(1, -1), [float(a @ y) + 0.02], 0.0, 1.0)
    assert r.lam[0] == 0.0 and r.outcome[0] == "inactive"


@pytest.mark.parametrize("seed", range(6))
def test_equality_rows_brute_force(seed):
    """Equality rows against enumeration of element states and active sets
    in which every equality row is held (tiny n)."""
    rng = np.random.default_rng(60 + seed)
    n, m = 6, 1 + seed % 2
    y = rng.uniform(-0.3, 1.3, n)
    A = rng.standard_normal((m, n))
    xs = rng.uniform(0.1, 0.9, n)
    b = A @ xs + rng.uniform(-0.3, 0.3, m)          # reachable targets, either side of A.clip(y)
    eq = np.array([True] + [bool(rng.integers(0, 2)) for _ in range(m - 1)])
    kappa = [0.0, 0.3][seed % 2]
    C = math.inf if kappa == 0.0 else 2.0 / kappa
    kind = "single" if m == 1 else "coupled"
    r = oracle.project(kind, y, A, b, 0.0, 1.0, C, eq=eq)
    surv = P.brute_force(y, A, b, 0.0, 1.0, kappa, eq=eq)
    assert surv, "no KKT point found by enumeration"
    for xb in surv:
        np.testing.assert_allclose(r.x, xb, atol=1e-8)
    cert = P.kkt_certificate(y, A, b, 0.0, 1.0, kappa, r.lam, r.x, eq=eq)
    assert cert["max"] < 1e-9, cert
    for j in np.flatnonzero(eq):
        assert abs(r.resid[j] - kappa * r.lam[j]) < 1e-9


def test_equality_row_is_two_opposite_inequalities():
    """Unregularized, {a.x = b} is {a.x <= b} and {-a.x <= -b} together: the
    projections coincide (enumeration over the two-row form)."""
    rng = np.random.default_rng(71)
    n = 7
    for _ in range(4):
        y = rng.uniform(-0.3, 1.3, n)
        a = rng.standard_normal(n)
        b = float(a @ rng.uniform(0.1, 0.9, n))
        r = oracle.project("single", y, a.reshape(1, -1), [b], 0.0, 1.0, eq=[True])
        surv = P.brute_force(y, np.vstack([a, -a]), np.array([b, -b]), 0.0, 1.0, 0.0)
        assert surv
        for xb in surv:
            np.testing.assert_allclose(r.x, xb, atol=1e-8)


def test_equality_blocks_are_separate_rows():
    """Independent blocks with equality flags = each block projected alone."""
    p = I.multi_material(3, fields=3, n_per=4000)
    eq = [True, False, True]
    b = p.b.copy()
    b[0] *= 1.5                                      # above a.clip(y) for the first field
    r = oracle.project("independent", p.y, p.A, b, p.lo, p.hi, offsets=p.offsets, eq=eq)
    for j in range(3):
        s, e = int(p.offsets[j]), int(p.offsets[j + 1])
        lj, _ = P.exact_single(p.y[s:e], p.A[s:e], b[j], p.lo, p.hi, 0.0, eq=eq[j])
        assert r.lam[j] == lj
    assert r.resid[0] == pytest.approx(0.0, abs=1e-12 * abs(b[0]) + 1e-15)


@pytest.mark.parametrize("seed", [0, 1])
def test_kkt_certificates_of_workloads(seed):
    """Every workload class is certified by the KKT residuals (eq. rkkt1-rkkt11)."""
    cases = [I.volume_2d(seed, vf=0.4), I.compliance_3d(seed, n=40000),
             I.multi_material(seed, n_per=20000), I.volume_com(seed, grid=(32, 16, 16))]
    for p in cases:
        r = oracle.project(p.kind, p.y, p.A, p.b, p.lo, p.hi, p.C, p.offsets)
        A = p.dense_rows()
        cert = P.kkt_certificate(p.y, A, p.b, p.lo, p.hi, r.kappa, r.lam, r.x)
        assert cert["max"] <= 1e-12, (p.meta, cert)


def test_planted_mistakes_are_caught(monkeypatch):
    """A plausible mistake in the oracle (wrong sign of A^T lam, dropped
    regularization term, transposed index) fails a pin."""
    case = json.load(open(GOLD))["cases"][1]
    y, A, b = np.array(case["y"]), np.array(case["A"]), np.array(case["b"])

    def wrong_sign(y_, A_, lam, lo, hi):
        A_ = np.atleast_2d(np.asarray(A_, float))
        z = np.asarray(y_, float) + A_.T @ np.asarray(lam, float)
        return np.clip(z, lo, hi), z

    with monkeypatch.context() as mp:
        mp.setattr(P, "clip_map", wrong_sign)
        r = oracle.project("coupled", y, A, b, 0.0, 1.0)
        assert not np.allclose(r.x, case["x"], atol=1e-6)

    # dropped kappa in h: the regularized golden case must fail
    case_r = json.load(open(GOLD))["cases"][2]
    lam_bad = P.coupled(y, A, b, 0.0, 1.0, 0.0)
    assert not np.allclose(lam_bad, case_r["lam"], atol=1e-6)
    # transposed operand: certificate of a perturbed multiplier is not clean
    cert = P.kkt_certificate(y, A, b, 0.0, 1.0, 0.0, np.array(case["lam"])[::-1])
    assert cert["max"] > 1e-3


def test_generators_shape_and_recipe():
    p = I.compliance_3d(0, n=200000)
    r = oracle.project(p.kind, p.y, p.A, p.b, p.lo, p.hi)
    assert 0.35 < r.n_free / p.n < 0.45          # b planted for ~40 % free
    assert r.lam[0] == pytest.approx(p.meta["planted_lambda"], rel=1e-3)
    q = I.volume_com(1, grid=(24, 12, 12))
    assert not q.meta["feasible"]
    assert q.A.shape == (5, 24 * 12 * 12) and q.A.dtype == np.float32


# ---------------------------------------------------------------- kappa path (Appendix A.2, choosing C)

@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("m", [1, 2, 3])
def test_kappa_path_trades_violation_for_distance(seed, m):
    """Along increasing C (a heavier penalty 1/kappa on the slack), the
    penalized problem min 1/2|x - y|^2 + 1/(2 kappa) |(Ax - b)_+|^2 can only
    lower the violation norm and raise the distance (the monotonicity of a
    quadratic penalty method); each point equals the enumerated solution of
    its own kappa (brute force), so the path is pinned point by point."""
    rng = np.random.default_rng(500 + 10 * seed + m)
    n = 6 if m < 3 else 5
    y, A, b = _random_case(rng, n, m, "infeasible")
    kind = "coupled" if m > 1 else "single"
    Cs = [2.0, 20.0, 200.0, 2e3, 2e4]
    pts = oracle.kappa_path(kind, y, A, b, 0.0, 1.0, Cs)
    for p in pts:
        sv = P.brute_force(y, A, b, 0.0, 1.0, p["kappa"])
        np.testing.assert_allclose(p["result"].x, sv[0], atol=1e-8)
        assert p["dist"] == pytest.approx(math.sqrt(P.fsum((sv[0] - y) ** 2)), abs=1e-7)
    for p, q in zip(pts, pts[1:]):
        assert q["violation_norm"] <= p["violation_norm"] + 1e-9
        assert q["dist"] >= p["dist"] - 1e-9
    # the infeasible row stays violated; the slack kappa lam_j is the
    # violation the regularized optimum keeps: kappa lam_j = (a_j.x - b_j)_+
    for p in pts:
        np.testing.assert_allclose(p["slack"], p["violation"], atol=1e-7)


def test_kappa_path_single_row_closed_form():
    """One infeasible row: every point is the saturated x with
    lam = (a.x_sat - b)/kappa, so the violation is constant and the distance
    too (hand-checkable; the slack equals the violation at every C)."""
    rng = np.random.default_rng(23)
    n = 300
    y = rng.uniform(-0.5, 1.5, n)
    a = rng.uniform(0.1, 1.0, n)
    lo, hi = 0.1, 1.0
    x_sat = np.full(n, lo)
    gap = 3.0
    b = P.fsum(a * x_sat) - gap
    pts = oracle.kappa_path("single", y, a.reshape(1, n), [b], lo, hi, [1e2, 1e4, 1e6], tau=0.5)
    d_sat = math.sqrt(P.fsum((x_sat - y) ** 2))
    for p in pts:
        assert p["lam"][0] == pytest.approx(gap / p["kappa"], rel=1e-12)
        assert p["max_violation"] == pytest.approx(gap, rel=1e-12)
        assert p["violation_over_tau"] == pytest.approx(gap / 0.5, rel=1e-12)
        assert p["dist"] == pytest.approx(d_sat, rel=1e-12)


# ---------------------------------------------------------------- many coupled rows (Alg. 2 at m = 32, 64)

@pytest.mark.parametrize("m,seed", [(32, 0), (32, 1), (64, 2), (64, 3)])
def test_planted_duals_recovered_many_rows(m, seed):
    """At m = 32 and 64 the oracle recovers the generator's planted multiplier
    (which satisfies the optimality conditions that close Appendix A.2 by
    construction, independently of the oracle), and both pass the KKT
    certificate.  The plant is exact for b up to the float64 rounding of its
    BLAS dot products, amplified by the conditioning of A D A^T."""
    p = I.many_rows(seed, m=m, grid=(24, 16, 16))
    A = p.A.astype(np.float64)
    lam_star = p.meta["planted_lambda"]
    kappa = 2.0 / p.C
    cert_star = P.kkt_certificate(p.y, A, p.b, p.lo, p.hi, kappa, lam_star)
    assert cert_star["max"] <= 1e-13
    r = oracle.project("coupled", p.y, p.A, p.b, p.lo, p.hi, p.C)
    np.testing.assert_allclose(r.lam, lam_star, rtol=0, atol=1e-7 * np.max(np.abs(lam_star)))
    cert = P.kkt_certificate(p.y, A, p.b, p.lo, p.hi, kappa, r.lam, r.x)
    assert cert["max"] <= 1e-12
    assert np.count_nonzero(r.lam) == np.count_nonzero(lam_star)


def test_planted_many_rows_equalities_and_single_active():
    """Equality rows keep multipliers of either sign (Sec. 3.2); with one
    active row the multiplier is that row's own 1-row solution (Alg. 2's
    Stage-1 exit), which the 1-row oracle computes independently."""
    p = I.many_rows(7, m=32, grid=(24, 16, 16), eq_rows=(1, 8, 19))
    eq = [bool((p.meta["eq_mask"] >> j) & 1) for j in range(p.m)]
    r = oracle.project("coupled", p.y, p.A, p.b, p.lo, p.hi, p.C, eq=eq)
    lam_star = p.meta["planted_lambda"]
    assert np.any(lam_star[np.array(eq)] < 0)
    np.testing.assert_allclose(r.lam, lam_star, rtol=0, atol=1e-7 * np.max(np.abs(lam_star)))
    q = I.many_rows(8, m=40, grid=(24, 16, 16), active=[5])
    r1 = oracle.project("coupled", q.y, q.A, q.b, q.lo, q.hi, q.C)
    ls, _ = P.exact_single(q.y, q.A[5].astype(np.float64), q.b[5], q.lo, q.hi, 2.0 / q.C)
    assert np.count_nonzero(r1.lam) == 1
    assert r1.lam[5] == pytest.approx(ls, rel=1e-9)


def test_planted_many_rows_catches_a_dropped_row():
    """A plausible mistake -- one row of A^T lam dropped from the clip map --
    breaks the certificate of the planted multiplier at m = 64."""
    p = I.many_rows(9, m=64, grid=(24, 16, 16))
    A = p.A.astype(np.float64)
    lam_star = p.meta["planted_lambda"]
    bad = lam_star.copy()
    bad[np.flatnonzero(lam_star)[3]] = 0.0
    cert = P.kkt_certificate(p.y, A, p.b, p.lo, p.hi, 2.0 / p.C, bad)
    assert cert["max"] > 1e-6
