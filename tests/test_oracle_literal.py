"""Pins for the paper-literal algorithms and the Alg. 3 step rules in the oracle."""
import math

import numpy as np
import pytest

import oracle
from oracle import projection as P
from oracle import literal
from oracle.pgd import PgdParams, cg_beta, step_size, pgd_step
from paper_2511_13905_amd import inputs as I


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_alg2_literal_reaches_the_certified_projection(seed):
    """Algorithm 2 as printed (absolute tol_N = 1e-6) converges to the unique
    regularized projection, to within what its tolerance allows."""
    p = I.volume_com(seed, grid=(32, 16, 16))
    r = oracle.project(p.kind, p.y, p.A, p.b, p.lo, p.hi, p.C)
    out = literal.alg2_newton(p.y.astype(float), p.A.astype(float), p.b, p.lo, p.hi, p.C)
    x, _ = P.clip_map(p.y, p.A, -out["y"], p.lo, p.hi)
    assert out["branch"] in ("stage1", "newton")
    assert np.max(np.abs(x - r.x)) < 5e-5


def test_alg2_literal_stage1_exit_on_single_active_row():
    """If one row alone is active, Stage 1 returns it without Newton (Sec. 3.2.3)."""
    rng = np.random.default_rng(2)
    n = 4000
    y = rng.uniform(-0.2, 1.2, n)
    a0 = np.full(n, 1.0 / n)
    a1 = rng.standard_normal(n) / n
    b = np.array([0.3, float(a1 @ np.clip(y, 0, 1)) + 1.0])    # row 1 far from active
    out = literal.alg2_newton(y, np.stack([a0, a1]), b, 0.0, 1.0, 1e12)
    assert out["branch"] == "stage1" and out["candidate"] == 0
    r = oracle.project("coupled", y, np.stack([a0, a1]), b, 0.0, 1.0, 1e12)
    x, _ = P.clip_map(y, np.stack([a0, a1]), -out["y"], 0.0, 1.0)
    assert np.max(np.abs(x - r.x)) < 1e-7


def test_step_size_rules():
    """Alg. 3 step rule: fallback at t = 0 and after warm-up on violation,
    otherwise eq. (final_alpha) with eps_alpha."""
    p = PgdParams()
    rho = np.array([0.5, 0.5, 0.5])
    grad = np.array([1.0, -4.0, 2.0])
    rho_prev = np.array([0.4, 0.6, 0.5])
    grad_prev = np.array([0.5, -3.0, 2.0])
    # t = 0: alpha = min(alpha_max, 0.2 / ||grad||_inf)
    a, fb = step_size(rho, rho_prev, grad, grad_prev, [0.0], [1.0], 0, p)
    assert fb and a == pytest.approx(0.2 / 4.0)
    # spectral branch: s = (0.1,-0.1,0), y = (0.5,-1,0): s.y = 0.15 > eps, s.s = 0.02
    a, fb = step_size(rho, rho_prev, grad, grad_prev, [0.0], [1.0], 10, p)
    lip = math.sqrt(0.02) / math.sqrt(1.25)
    assert not fb and a == pytest.approx(min(0.02 / 0.15, 2 * lip, p.alpha_max))
    # s.y <= eps: Lipschitz estimate of eq. (alpha)
    grad_prev2 = np.array([1.5, -5.0, 2.0])        # y = (-0.5, 1, 0): s.y = -0.15
    a, fb = step_size(rho, rho_prev, grad, grad_prev2, [0.0], [1.0], 10, p)
    assert not fb and a == pytest.approx(min(lip, p.alpha_max))
    # after warm-up, a violated constraint triggers the fallback
    a, fb = step_size(rho, rho_prev, grad, grad_prev, [1.1], [1.0], 60, p)
    assert fb and a == pytest.approx(0.05)
    # ... but not before warm-up
    a, fb = step_size(rho, rho_prev, grad, grad_prev, [1.1], [1.0], 49, p)
    assert not fb
    # cap at alpha_max
    a, fb = step_size(rho, rho_prev, np.full(3, 1e-6), np.full(3, 1e-6), [0.0], [1.0], 0, p)
    assert a == p.alpha_max


def test_cg_beta_rules():
    """eq. (CG): Polak-Ribiere with restart at 0; Fletcher-Reeves option."""
    g = np.array([1.0, 2.0])
    gp = np.array([2.0, 0.0])
    # PR: g.(g - gp) / |gp|^2 = (1*-1 + 2*2)/4 = 0.75
    assert cg_beta(g, gp, 5, "pr+") == pytest.approx(0.75)
    # restart: g.(g-gp) < 0 -> 0
    assert cg_beta(np.array([1.0, 0.0]), np.array([3.0, 0.0]), 5, "pr+") == 0.0
    assert cg_beta(g, gp, 5, "fr") == pytest.approx(5.0 / 4.0)
    assert cg_beta(g, gp, 0, "pr+") == 0.0


def test_pgd_step_inactive_is_clipped_gradient_step():
    """With the constraint slack, rho_{t+1} = clip(rho_t + omega alpha d_t)."""
    rng = np.random.default_rng(4)
    n = 1000
    rho = rng.uniform(0.2, 0.8, n)
    grad = rng.standard_normal(n)
    A = np.full((1, n), 1.0 / n)
    out = pgd_step("single", rho, rho, grad, grad, -grad, A, [0.5], [0.99], 0, 1e-3, 1.0)
    alpha = 0.2 / np.max(np.abs(grad))
    assert out["alpha"] == pytest.approx(alpha)
    np.testing.assert_allclose(out["x"], np.clip(rho - alpha * grad, 1e-3, 1.0), atol=1e-15)
    assert out["proj"].outcome == ["inactive"]


def test_pgd_step_rhs_matches_paper_form():
    """With omega = 1 and d = -grad f, b_j - a_j.rho~ equals the paper's
    G-hat = G - g + alpha grad f . grad g (eq. h / Appendix A.1)."""
    st = I.pgd_compliance_3d(0, t=0, n=5000)
    p = PgdParams(cg_rule="none")
    A = st.problem.A.astype(np.float64)
    out = pgd_step("single", st.rho, st.rho_prev, st.grad, st.grad_prev, st.d_prev, A,
                   st.g, st.G, st.t, I.LO, I.HI, p=p)
    a = A[0]
    ghat = st.G[0] - st.g[0] + out["alpha"] * P.fsum(st.grad.astype(float) * a)
    assert out["b"][0] - P.fsum(a * out["rho_tilde"]) == pytest.approx(ghat, rel=1e-9, abs=1e-6)


# ------------------------------------------------------------------ hand-worked Algorithm 3 steps

def _golden_pgd():
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "pgd_step_hand_worked.json")
    with open(path) as f:
        return json.load(f)["cases"]


def _run_golden(c, pgd_fn=pgd_step):
    p = PgdParams(cg_rule=c["cg_rule"], omega=c["omega"], tol=c["tol"])
    sd = np.float32 if c.get("stream_dtype") == "float32" else None
    A = np.asarray(c["A"], dtype=np.float64)
    C = math.inf if c["C"] == "inf" else float(c["C"])
    f = lambda k: np.asarray(c[k], dtype=np.float64)
    return pgd_fn(c["kind"], f("rho"), f("rho_prev"), f("grad"), f("grad_prev"), f("d_prev"), A,
                  c["g"], c["G"], c["t"], c["lo"], c["hi"], C=C, p=p, stream_dtype=sd)


@pytest.mark.parametrize("name", [c["name"] for c in _golden_pgd()])
def test_pgd_step_hand_worked(name):
    """One body of Algorithm 3 against values worked by hand with exact
    fractions (tests/golden/pgd_step_hand_worked.json): the spectral step and
    the fallback after warm-up, beta of eq. (CG) in both rules with beta != 0,
    omega != 1 (Sec. 3.4.3), b, the projection and the stop test."""
    c = next(c for c in _golden_pgd() if c["name"] == name)
    out = _run_golden(c)
    assert out["used_fallback"] == c["used_fallback"]
    assert out["alpha"] == pytest.approx(c["alpha"], rel=1e-13)
    assert out["beta"] == pytest.approx(c["beta"], rel=1e-13, abs=1e-300)
    np.testing.assert_allclose(out["d"], c["d"], rtol=1e-13, atol=0)
    np.testing.assert_allclose(out["rho_tilde"], c["rho_tilde"], rtol=1e-13, atol=0)
    np.testing.assert_allclose(out["b"], c["b"], rtol=1e-13)
    assert out["proj"].outcome == [c["outcome"]]
    np.testing.assert_allclose(out["proj"].lam, c["lam"], rtol=1e-6 if c["lam"][0] < 1e-6 else 1e-12, atol=0)
    np.testing.assert_allclose(out["x"], c["x"], rtol=1e-12, atol=0)
    if "x_stored" in c:
        assert np.array_equal(out["x_stored"], np.asarray(c["x_stored"]))
    if c["rel_change"] == 0.0:
        assert out["rel_change"] == 0.0
    else:
        assert out["rel_change"] == pytest.approx(c["rel_change"], rel=1e-12)
    assert out["converged"] == c["converged"]
    if "rel_change_unrounded" in c:
        # the same step with float64 storage measures the unrounded iterate
        c64 = dict(c)
        c64.pop("stream_dtype")
        o64 = _run_golden(c64)
        assert o64["rel_change"] == pytest.approx(c["rel_change_unrounded"], rel=1e-6)


def test_pgd_step_planted_mistakes_fail_the_hand_worked_pins(monkeypatch):
    """Plausible slips in the Algorithm 3 body (a flipped beta sign, omega
    dropped, the stop test on the unrounded iterate, FR and PR+ swapped, the
    fallback ignored after warm-up) each change a value the hand-worked cases
    fix."""
    import oracle.pgd as PG
    cases = {c["name"]: c for c in _golden_pgd()}

    def fails(name, **patch):
        with monkeypatch.context() as mp:
            for k, v in patch.items():
                mp.setattr(PG, k, v)
            c = cases[name]
            out = _run_golden(c, PG.pgd_step)
            ok = (np.allclose(out["d"], c["d"], rtol=1e-12, atol=0)
                  and np.allclose(out["rho_tilde"], c["rho_tilde"], rtol=1e-12, atol=0)
                  and np.allclose(out["x"], c["x"], rtol=1e-12, atol=0)
                  and out["alpha"] == pytest.approx(c["alpha"], rel=1e-13)
                  and (out["rel_change"] == c["rel_change"] if c["rel_change"] == 0.0
                       else out["rel_change"] == pytest.approx(c["rel_change"], rel=1e-12)))
            return not ok

    real_beta = PG.cg_beta
    assert fails("spectral_step_pr_plus_half_omega", cg_beta=lambda *a, **k: -real_beta(*a, **k))
    swap = {"pr+": "fr", "fr": "pr+", "none": "none"}
    assert fails("fallback_after_warmup_fletcher_reeves_active_row",
                 cg_beta=lambda g, gp, t, rule="pr+": real_beta(g, gp, t, swap[rule]))
    assert fails("spectral_step_pr_plus_half_omega",
                 PgdParams=PgdParams, pgd_step=_omega_dropped(PG))
    real_step = PG.step_size
    assert fails("fallback_after_warmup_fletcher_reeves_active_row",
                 step_size=lambda rho, rp, gr, gp, g, G, t, p: real_step(rho, rp, gr, gp, g, G, min(t, 1), p))
    real_np = PG.np

    class NoRound:                      # the stop test on the unrounded iterate
        def __getattr__(self, k):
            return getattr(real_np, k)

        @staticmethod
        def dtype(v):
            return real_np.dtype(real_np.float64)
    assert fails("stop_test_on_the_stored_iterate", np=NoRound())


def _omega_dropped(PG):
    real = PG.pgd_step

    def wrapped(*a, p=None, **k):
        q = PgdParams(**{**p.__dict__, "omega": 1.0})
        return real(*a, p=q, **k)
    return wrapped
