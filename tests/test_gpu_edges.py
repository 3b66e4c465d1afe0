"""GPU parity on the edge cases of the method, through the C ABI.

Rows with zero coefficients, iteration limits that end a search or the
Newton stage early, a flat stretch of the unregularized dual (x unique,
lambda not), coupled rows without regularization, omega != 1 and the
fallback step after warm-up in Algorithm 3, equality-row outcomes on the
coupled path, and the error every result states against the exact
solution.  Every case prints its name and shape before touching the GPU.
"""
import dataclasses
import math

import numpy as np
import pytest

import oracle
from oracle import projection as P
from oracle.pgd import PgdParams
from paper_2511_13905_amd import inputs as I

from parity import check, free_from_mask

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2511_13905_amd.api import Context
    c = Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def say(*a):
    print("[case]", *a, flush=True)


def run(ctx, p, params=None, eq=None):
    y = dev(p.y)
    A = dev(p.A)
    mask = torch.zeros((p.n + 31) // 32, dtype=torch.int32, device="cuda:0")
    x, r = ctx.project(p.kind, y, A, p.b, p.lo, p.hi, p.C, offsets=p.offsets, free_mask=mask, params=params, eq=eq)
    torch.cuda.synchronize()
    return x.cpu().numpy(), r, free_from_mask(mask.cpu().numpy().view(np.uint32), p.n)


def orc(p, eq=None):
    return oracle.project(p.kind, p.y, p.A, p.b, p.lo, p.hi, p.C, p.offsets, eq=eq)


def f32_ulp(v):
    return np.spacing(np.abs(np.asarray(v, dtype=np.float32))).astype(np.float64)


# ------------------------------------------------------------------ zero coefficients

def _with_zeros(p, frac, seed):
    """A copy of p whose rows have a_ji = 0 on a random fraction of the elements
    (whole columns for coupled rows, plus extra zeros in row 1)."""
    rng = np.random.default_rng(seed)
    A = np.array(p.A, copy=True)
    cols = rng.random(p.n) < frac
    if A.ndim == 2:
        A[:, cols] = 0
        if A.shape[0] > 1:
            A[1, rng.random(p.n) < frac] = 0
    else:
        A[cols] = 0
    return dataclasses.replace(p, A=A)


@pytest.mark.parametrize("case", ["single-f32", "single-f64", "independent", "coupled", "coupled-infeasible"])
def test_zero_coefficients(ctx, case):
    """Elements with a_i = 0 have no breakpoint (left out of the bracket) and
    stay at clip(y_i) whatever the multiplier."""
    if case == "single-f32":
        p = _with_zeros(I.compliance_3d(5, n=300007), 0.2, 1)
    elif case == "single-f64":
        p = _with_zeros(I.volume_2d(6, nx=256, ny=129, vf=0.3), 0.3, 2)
    elif case == "independent":
        p = _with_zeros(I.multi_material(3, fields=4, n_per=50021), 0.25, 3)
    elif case == "coupled":
        p = _with_zeros(I.volume_com(0, grid=(64, 32, 16)), 0.2, 4)
    else:
        p = _with_zeros(I.volume_com(1, grid=(64, 32, 16)), 0.2, 5)
    say("zero coefficients", case, p.n)
    x, r, fm = run(ctx, p)
    ref = orc(p)
    check(p, x, r, ref, fm)
    A = p.dense_rows() if p.kind == "independent" else np.atleast_2d(p.A)
    zero = np.all(A == 0, axis=0)
    assert zero.any()
    yz = np.clip(p.y.astype(np.float64)[zero], p.lo, p.hi).astype(p.y.dtype)
    assert np.array_equal(x[zero], yz)


# ------------------------------------------------------------------ iteration limits

def test_search_iteration_limit(ctx):
    """max_search = 1: the 1-D search stops after one pass with outcome
    MAXITER; x is the clip map at the multiplier it returns."""
    for mode in ("newton", "bisect"):
        p = I.compliance_3d(7, n=200003)
        say("search limit", mode, p.n)
        from paper_2511_13905_amd.api import make_params
        x, r, fm = run(ctx, p, params=make_params(max_search=1, search=mode))
        assert r["outcome"] == "maxiter" and r["row_outcome"] == ["maxiter"]
        assert r["iters_search"] == 1
        xl, z = P.clip_map(p.y, p.A, r["lam"], p.lo, p.hi)
        assert np.all(np.abs(x.astype(np.float64) - xl) <= f32_ulp(xl))
        # the stated error covers the distance to the exact multiplier
        ref = orc(p)
        assert abs(r["lam"][0] - ref.lam[0]) <= r["lambda_err"][0]
        assert abs(r["lam"][0] - ref.lam[0]) <= r["lambda_width"]


def test_newton_iteration_limit(ctx):
    """max_newton = 1: the coupled solve stops after one Newton iteration
    with outcome MAXITER; x is the clip map at the multipliers it returns.
    Stage 1 is skipped (it would end the infeasible seed, whose single
    active row passes the candidate check)."""
    from paper_2511_13905_amd.api import make_params
    for seed in (0, 1):
        p = I.volume_com(seed, grid=(48, 24, 24))
        say("newton limit", seed, p.n)
        x, r, fm = run(ctx, p, params=make_params(max_newton=1, stage1=0))
        assert r["path"] == 3
        assert r["outcome"] == "maxiter" and r["iters_newton"] == 1
        assert all(o == "maxiter" for o in r["row_outcome"])
        xl, z = P.clip_map(p.y, p.A, r["lam"], p.lo, p.hi)
        assert np.all(np.abs(x.astype(np.float64) - xl) <= f32_ulp(xl))


# ------------------------------------------------------------------ flat stretch, kappa = 0

def test_kappa0_plateau(ctx):
    """One unregularized row whose dual function is zero on a whole interval
    of multipliers (every element saturated there): x is unique, lambda is
    any point of the interval.  x against the oracle (which returns the
    interval's left end) and lambda checked to lie in the interval."""
    k = 40000
    n = 3 * k
    rng = np.random.default_rng(11)
    lo, hi = I.LO, I.HI
    # evenly spaced values (shuffled): neighbouring breakpoints are 2.5e-6 n
    # apart, far above what the stop tolerance can leave unresolved
    grid = np.arange(k) / k
    g1 = 3.0 + rng.permutation(grid)            # at hi until lam/n >= y - 1 >= 2
    g2 = -0.5 + 0.5 * rng.permutation(grid)     # at lo throughout
    g3 = 0.5 + 0.1 * rng.permutation(grid)      # free at 0, at lo once lam/n >= y - lo
    y = np.concatenate([g1, g2, g3]).astype(np.float32)
    a = np.full(n, 1.0 / n, dtype=np.float32)
    xs = np.concatenate([np.full(n // 3, hi), np.full(2 * (n // 3), lo)])
    b = math.fsum((a.astype(np.float64) * xs).tolist())
    p = I.Problem("single", y, a.reshape(1, n), np.array([b]))
    say("kappa = 0 plateau", n)
    x, r, fm = run(ctx, p)
    ref = orc(p)
    check(p, x, r, ref, fm)
    np.testing.assert_array_equal(x, xs.astype(np.float32))
    left = float(np.max(g3.astype(np.float32).astype(np.float64) - lo)) * n
    right = float(np.min(g1.astype(np.float32).astype(np.float64) - hi)) * n
    assert left * (1 - 1e-6) <= r["lam"][0] <= right * (1 + 1e-12)
    h = P.h_map(p.y, p.A, p.b, r["lam"], lo, hi, 0.0)
    assert abs(h[0]) <= 1e-12 * P.row_scale(p.A, lo, hi)[0]


# ------------------------------------------------------------------ coupled, C = infinity

@pytest.mark.parametrize("seed", [0, 1])
def test_coupled_unregularized_full_rank(ctx, seed):
    """Three dense rows of full rank with C = INFINITY (kappa = 0): the
    unregularized problem of eq. (linearized), unique in x and lambda."""
    rng = np.random.default_rng(100 + seed)
    n = 90001
    y = (rng.uniform(0, 1, n) - 0.1 * rng.standard_normal(n)).astype(np.float32)
    rows = np.stack([np.full(n, 1.0 / n), rng.standard_normal(n) / n, (rng.uniform(0, 1, n) - 0.3) / n])
    A = rows.astype(np.float32)
    Ad = A.astype(np.float64)
    xc = np.clip(y.astype(np.float64), I.LO, I.HI)
    b = np.array([0.35, float(Ad[1] @ xc) - 0.02 * np.abs(Ad[1]).sum(), float(Ad[2] @ xc) - 0.01 * np.abs(Ad[2]).sum()])
    p = I.Problem("coupled", y, A, b, C=math.inf)
    say("coupled kappa = 0", seed, n)
    x, r, fm = run(ctx, p)
    ref = orc(p)
    assert P.kkt_certificate(p.y, p.A, p.b, p.lo, p.hi, 0.0, ref.lam, ref.x)["max"] <= 1e-10
    assert np.count_nonzero(ref.lam > 0) >= 2
    check(p, x, r, ref, fm)
    assert r["kappa"] == 0.0
    np.testing.assert_allclose(r["lam"], ref.lam, rtol=1e-7, atol=1e-9 * float(np.max(np.abs(ref.lam))))


# ------------------------------------------------------------------ equality row outcome, coupled

def test_coupled_equality_row_outcome(ctx):
    """A coupled equality row whose multiplier is negative (the row is
    lifted to its target) is reported converged, as on the 1-D path."""
    p = I.volume_com(0, grid=(96, 48))
    p = dataclasses.replace(p, b=p.b.copy())
    p.b[0] = 0.45 * float(np.sum(p.A[0].astype(np.float64)))
    eq = [True, False, False, False, False]
    say("coupled equality outcome", p.n)
    x, r, fm = run(ctx, p, eq=eq)
    ref = orc(p, eq=eq)
    check(p, x, r, ref, fm)
    assert r["lam"][0] < 0.0
    assert r["row_outcome"][0] == "converged"
    assert r["outcome"] in ("converged", "inactive")
    # the same row set at an unreachable level is infeasible from above
    q = dataclasses.replace(p, b=p.b.copy())
    q.b[0] = 1.5 * float(np.sum(p.A[0].astype(np.float64)))
    say("coupled equality infeasible", q.n)
    x, r, fm = run(ctx, q, eq=eq)
    assert r["row_outcome"][0] == "infeasible" and r["outcome"] == "infeasible"


# ------------------------------------------------------------------ Algorithm 3 edges

def _pgd_inputs(n, seed):
    rng = np.random.default_rng(seed)
    rho = np.clip(rng.uniform(0, 1, n), I.LO, I.HI).astype(np.float32)
    grad = rng.standard_normal(n).astype(np.float32)
    rho_prev = (rho - 0.01 * rng.standard_normal(n)).astype(np.float32)
    # grad.(grad - grad_prev) > 0, so that PR+ keeps beta > 0
    grad_prev = (0.8 * grad + 0.1 * rng.standard_normal(n)).astype(np.float32)
    d_prev = (-grad_prev + 0.05 * rng.standard_normal(n)).astype(np.float32)
    return rho, rho_prev, grad, grad_prev, d_prev


def _pgd_compare(ctx, kind, A, g, G, t, C, hyper, seed, n):
    rho, rho_prev, grad, grad_prev, d_prev = _pgd_inputs(n, seed)
    d = dev(d_prev)
    kw = {k: v for k, v in hyper.items()}
    x, out = ctx.pgd_step(kind, dev(A), dev(rho), dev(rho_prev), dev(grad), dev(grad_prev), d, g(rho), G, t,
                          I.LO, I.HI, C=C, **kw)
    torch.cuda.synchronize()
    ref = oracle.pgd_step(kind, rho, rho_prev, grad, grad_prev, d_prev, A, g(rho), G, t, I.LO, I.HI, C=C,
                          p=PgdParams(**{k: v for k, v in hyper.items() if k in ("omega", "cg_rule", "tol")}),
                          stream_dtype=np.float32)
    assert out["used_fallback"] == ref["used_fallback"]
    assert out["alpha"] == pytest.approx(ref["alpha"], rel=1e-12)
    assert out["beta"] == pytest.approx(ref["beta"], rel=1e-9, abs=1e-15)
    np.testing.assert_allclose(d.cpu().numpy(), ref["d"], rtol=1e-6, atol=1e-7)
    prob = I.Problem(kind, ref["rho_tilde"], A, ref["b"], C=C)
    check(prob, x.cpu().numpy(), out["proj"], ref["proj"])
    assert out["rel_change"] == pytest.approx(ref["rel_change"], rel=1e-5)
    assert out["converged"] == ref["converged"]
    return out, ref


@pytest.mark.parametrize("kind", ["single", "coupled"])
def test_pgd_step_omega_half(ctx, kind):
    """rho~ = rho_t + omega alpha_t d_t with omega = 0.5 (Alg. 3, Sec. 3.4.3)."""
    if kind == "single":
        base = I.compliance_3d(8, n=150001)
        A, C = base.A, math.inf
        G = np.array([base.b[0]])
    else:
        base = I.volume_com(0, grid=(48, 24, 24))
        A, C = base.A, base.C
        G = base.b.copy()
    Ad = np.atleast_2d(A.astype(np.float64))
    say("pgd omega 0.5", kind, base.n)
    out, ref = _pgd_compare(ctx, kind, A, lambda r: Ad @ r.astype(np.float64), G, 70, C,
                            {"omega": 0.5, "cg_rule": "pr+"}, 21, base.n)
    assert out["beta"] > 0.0


@pytest.mark.parametrize("kind", ["single", "coupled"])
def test_pgd_step_fallback_after_warmup(ctx, kind):
    """Past warm-up a violated constraint (g_j - G_j > tol_N) takes the
    fallback step alpha = min(alpha_max, alpha_fb / ||grad f||_inf) (Alg. 3)."""
    if kind == "single":
        base = I.compliance_3d(9, n=150001)
        A, C = base.A, math.inf
    else:
        base = I.volume_com(0, grid=(48, 24, 24))
        A, C = base.A, base.C
    Ad = np.atleast_2d(A.astype(np.float64))
    rho = _pgd_inputs(base.n, 22)[0]
    gval = Ad @ rho.astype(np.float64)
    G = gval - 1e-3 * np.maximum(np.abs(gval), 1e-3)        # every row violated by 0.1%
    say("pgd fallback after warm-up", kind, base.n)
    out, ref = _pgd_compare(ctx, kind, A, lambda r: Ad @ r.astype(np.float64), G, 60, C,
                            {"cg_rule": "pr+"}, 22, base.n)
    assert out["used_fallback"] and ref["used_fallback"]
    grad = _pgd_inputs(base.n, 22)[2].astype(np.float64)
    assert out["alpha"] == pytest.approx(min(100.0, 0.2 / np.max(np.abs(grad))), rel=1e-12)


# ------------------------------------------------------------------ stated error

STATED = {
    "single-f32": lambda: I.compliance_3d(12, n=400009),
    "single-f64": lambda: I.volume_2d(3, nx=128, ny=64, vf=0.4),
    "single-infeasible": lambda: dataclasses.replace(I.compliance_3d(13, n=100003), b=np.array([-1e9])),
    "independent": lambda: I.multi_material(5, fields=4, n_per=65537),
    "coupled": lambda: I.volume_com(2, grid=(64, 32, 16)),
    "coupled-infeasible": lambda: I.volume_com(3, grid=(64, 32, 16)),
    "coupled-stage1": lambda: I.volume_com(0, grid=(64, 32, 16), target=(0.5, 0.25), band=(0.3, 0.2)),
}


@pytest.mark.parametrize("case", list(STATED))
def test_stated_error_covers_the_oracle_error(ctx, case):
    """Every result states a bound on its error (pgdto_result.lambda_err,
    x_err, res_inf): it must be at least the error measured against the
    float64 oracle."""
    p = STATED[case]()
    say("stated error", case, p.n)
    x, r, fm = run(ctx, p)
    ref = orc(p)
    check(p, x, r, ref, fm)
    xerr = float(np.max(np.abs(x.astype(np.float64) - ref.x)))
    print("x error", xerr, "stated", r["x_err"], "lambda", r["lam"], "stated", r["lambda_err"],
          "res_inf", r["res_inf"], "width", r["lambda_width"], flush=True)
    assert xerr <= r["x_err"]
    assert r["x_err"] < 1e-3
    for j in range(p.m):
        assert abs(r["lam"][j] - ref.lam[j]) <= r["lambda_err"][j], j
    assert math.isfinite(r["res_inf"]) and r["res_inf"] >= 0.0
    if not case.endswith("infeasible") or p.C != math.inf:
        assert r["res_inf"] <= 1e-6
    if case.startswith("single") and r["path"] == 1:
        assert abs(r["lam"][0] - ref.lam[0]) <= r["lambda_width"]
