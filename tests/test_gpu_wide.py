"""GPU parity of the wide coupled kernel (9 to 64 dense rows, Alg. 2 with the
Jacobian sums A D A^T of eq. reg_jacobian on the matrix cores) against the
CPU oracle and against the planted multipliers of the generator.

Every case prints its name, seed and shape before touching the GPU.
"""
import math
import os

import numpy as np
import pytest

import oracle
from oracle import projection as P
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


def run(ctx, p, params=None, eq=None, lam0=None, C=None):
    mask = torch.zeros((p.n + 31) // 32, dtype=torch.int32, device="cuda:0")
    x, r = ctx.project(p.kind, dev(p.y), dev(p.A), p.b, p.lo, p.hi, p.C if C is None else C, free_mask=mask,
                       params=params, eq=eq, lam0=lam0)
    torch.cuda.synchronize()
    return x.cpu().numpy(), r, free_from_mask(mask.cpu().numpy().view(np.uint32), p.n)


def eq_flags(p):
    em = p.meta.get("eq_mask", 0)
    return [bool((em >> j) & 1) for j in range(p.m)] if em else None


def orc(p, C=None):
    return oracle.project(p.kind, p.y, p.A, p.b, p.lo, p.hi, p.C if C is None else C, eq=eq_flags(p))


def lam_close(r, ref, planted=None):
    g = np.asarray(r["lam"])
    scale = max(1.0, float(np.max(np.abs(ref.lam))))
    assert np.max(np.abs(g - ref.lam)) <= 1e-6 * scale, (g[:8], ref.lam[:8])
    # the stated error covers the difference to the oracle (plus the oracle's own rounding)
    err = np.abs(g - ref.lam)
    assert np.all(err <= np.asarray(r["lambda_err"]) + 1e-9 * scale), (err.max(), min(r["lambda_err"]))
    if planted is not None:
        assert np.max(np.abs(g - planted)) <= 1e-6 * scale


@pytest.mark.parametrize("m,grid,seed", [(9, (24, 16, 16), 0), (16, (25, 17, 15), 1), (17, (24, 16, 16), 2),
                                         (32, (25, 17, 15), 3), (48, (24, 16, 16), 4), (64, (25, 17, 15), 5),
                                         (64, (24, 16, 16), 6)])
def test_wide_planted(ctx, m, grid, seed):
    """Planted multipliers on every fourth row, several tiles and a ragged last chunk."""
    p = I.many_rows(seed, m=m, grid=grid)
    say("wide planted", m, grid, seed, p.n)
    x, r, fm = run(ctx, p)
    ref = orc(p)
    assert r["error"] == 0 and r["outcome"] == "converged", r["outcome"]
    check(p, x, r, ref, fm)
    lam_close(r, ref, p.meta["planted_lambda"])
    # the KKT residuals of the returned multiplier, recomputed in float64
    cert = P.kkt_certificate(p.y, p.A.astype(np.float64), p.b, p.lo, p.hi, r["kappa"], np.asarray(r["lam"]))
    assert cert["primal"] <= 1e-10 and cert["compl"] <= 1e-10, cert
    # of x as stored: up to the rounding of x to float32 (2^-24 sigma_j)
    assert r["res_inf"] <= 2.0 ** -24
    assert r["n_free"] == ref.n_free
    print("path", r["path"], "passes", r["passes"], "newton", r["iters_newton"], "ls", r["iters_ls"], flush=True)


def test_wide_many_tiles(ctx):
    """m = 64 over 30 tiles of 4096 elements."""
    p = I.many_rows(11, m=64, grid=(64, 48, 40))
    say("wide many tiles", p.m, p.n)
    x, r, fm = run(ctx, p)
    ref = orc(p)
    check(p, x, r, ref, fm)
    lam_close(r, ref, p.meta["planted_lambda"])


def test_wide_stage1_exit(ctx):
    """One active row: its Stage-1 multiplier satisfies every row, so the
    float64 candidate check (matrix cores) ends the solve (path 2)."""
    p = I.many_rows(12, m=40, grid=(24, 16, 16), active=[5])
    say("wide stage-1 exit", p.m, p.n)
    x, r, fm = run(ctx, p)
    ref = orc(p)
    check(p, x, r, ref, fm)
    lam_close(r, ref, p.meta["planted_lambda"])
    assert r["path"] == 2 and r["iters_newton"] == 0
    assert [j for j, l in enumerate(r["lam"]) if l != 0.0] == [5]


def test_wide_candidates_beyond_one_check_pass(ctx):
    """More than 16 rows violated at lam = 0 and an active row past the first
    16 candidates: the check runs in several passes, in row order."""
    p = I.many_rows(13, m=64, grid=(24, 16, 16), active=[45], margin=1e-3)
    h0 = P.h_map(p.y, p.A.astype(np.float64), p.b, np.zeros(p.m), p.lo, p.hi, 2.0 / p.C)
    say("wide multi-check", p.m, int(np.sum(h0 > 0)))
    x, r, fm = run(ctx, p)
    ref = orc(p)
    check(p, x, r, ref, fm)
    lam_close(r, ref, p.meta["planted_lambda"])


def test_wide_equality_rows(ctx):
    """Equality rows (Sec. 3.2) with multipliers of either sign."""
    p = I.many_rows(14, m=32, grid=(24, 16, 16), eq_rows=(1, 8, 19))
    say("wide equality rows", p.m, p.meta["eq_mask"])
    x, r, fm = run(ctx, p, eq=eq_flags(p))
    ref = orc(p)
    check(p, x, r, ref, fm)
    lam_close(r, ref, p.meta["planted_lambda"])
    assert any(l < 0.0 for l in r["lam"])


@pytest.mark.parametrize("params", [{"stage1": 0}, {"ncp": "paper"}, {"search": "bisect"}])
def test_wide_variants(ctx, params):
    p = I.many_rows(15, m=24, grid=(24, 16, 16))
    say("wide variant", params)
    x, r, fm = run(ctx, p, params=params)
    ref = orc(p)
    check(p, x, r, ref, fm)
    lam_close(r, ref)


def test_wide_warm_start(ctx):
    """Newton from the solution's multipliers stops at once."""
    p = I.many_rows(16, m=48, grid=(24, 16, 16))
    ref = orc(p)
    say("wide warm start", p.m)
    _, cold, _ = run(ctx, p)
    x, warm, fm = run(ctx, p, lam0=list(ref.lam))
    check(p, x, warm, ref, fm)
    lam_close(warm, ref)
    assert warm["passes"] < cold["passes"] and warm["iters_newton"] <= 1


@pytest.mark.parametrize("tau", [1e-4, 1e-7])
def test_wide_automatic_penalty(ctx, tau):
    """C < 0: kappa = tau / (largest breakpoint), Appendix A.2."""
    p = I.many_rows(17, m=20, grid=(24, 16, 16))
    A = p.A.astype(np.float64)
    C = P.auto_C("coupled", p.y, A, p.lo, p.hi, tau)
    say("wide auto C", tau, C)
    x, r, fm = run(ctx, p, C=-tau)
    ref = orc(p, C=C)
    assert r["kappa"] == pytest.approx(2.0 / C, rel=1e-12)
    check(p, x, r, ref, fm)
    lam_close(r, ref)


def test_wide_infeasible_row(ctx):
    """A row that cannot hold on the box: kappa > 0 gives the regularized
    answer with positive slack (infeasible row outcome)."""
    p = I.many_rows(18, m=12, grid=(24, 16, 16))
    A = p.A.astype(np.float64)
    p.b[3] = float(np.sum(np.where(A[3] > 0, p.lo * A[3], p.hi * A[3]))) - 1e-3 * abs(p.b[3] + 1e-12)
    p.C = 1e8
    say("wide infeasible row", p.m)
    x, r, fm = run(ctx, p)
    ref = orc(p)
    check(p, x, r, ref, fm)
    lam_close(r, ref)
    assert r["row_outcome"][3] == "infeasible" and r["slack"][3] > 0.0


def test_wide_inactive_and_grid_invariance(ctx):
    """All rows inactive: x = clip(y) bit for bit; and a 5-workgroup grid
    gives the bits of the full grid (reduction orders follow the tiles)."""
    from paper_2511_13905_amd.api import Context
    p = I.many_rows(19, m=33, grid=(40, 32, 24))
    q = I.many_rows(19, m=33, grid=(40, 32, 24))
    q.b = q.b + 10.0 * P.row_scale(q.A.astype(np.float64), q.lo, q.hi)
    say("wide inactive / grid", p.n)
    x, r, _ = run(ctx, q)
    assert r["outcome"] == "inactive" and r["path"] == 0 and all(l == 0.0 for l in r["lam"])
    assert np.array_equal(x, np.clip(q.y, np.float32(q.lo), np.float32(q.hi)))
    os.environ["PGDTO_GRID"] = "5"
    try:
        c5 = Context(0)
    finally:
        del os.environ["PGDTO_GRID"]
    try:
        x0, r0, m0 = run(ctx, p)
        x1, r1, m1 = run(c5, p)
        g0, _ = ctx.last_launch()
        g1, _ = c5.last_launch()
        assert g1 == 5 and g0 > 5
        assert np.array_equal(x0, x1) and np.array_equal(m0, m1)
        assert r0["lam"] == r1["lam"] and r0["passes"] == r1["passes"]
    finally:
        c5.close()


@pytest.mark.parametrize("m", [32, 64])
def test_wide_full_size(ctx, m):
    """256 x 128 x 128 elements: the multipliers against the planted ones,
    sampled x against clip(y - A^T lam) in float64 with the GPU's lam."""
    p = I.many_rows(20 + m, m=m)
    say("wide full size", m, p.n)
    x, r, fm = run(ctx, p)
    assert r["error"] == 0 and r["outcome"] == "converged"
    lam = np.asarray(r["lam"])
    planted = p.meta["planted_lambda"]
    assert np.max(np.abs(lam - planted)) <= 1e-6 * np.max(np.abs(planted))
    assert r["res_inf"] <= 2.0 ** -24
    rng = np.random.default_rng(m)
    idx = rng.choice(p.n, 4096, replace=False)
    z = p.y[idx].astype(np.float64) - lam @ p.A[:, idx].astype(np.float64)
    xe = np.clip(z, p.lo, p.hi)
    assert np.max(np.abs(x[idx] - xe) / np.maximum(np.abs(xe), 1e-3)) <= 2e-6
    free = (z >= p.lo) & (z <= p.hi)
    far = np.minimum(np.abs(z - p.lo), np.abs(z - p.hi)) > 1e-6
    assert np.array_equal(fm[idx][far], free[far])
    print("passes", r["passes"], "newton", r["iters_newton"], "ls", r["iters_ls"], "path", r["path"], flush=True)


def test_wide_routes_that_stay_small(ctx):
    """Beyond 8 rows: float64 streams, Algorithm 3 steps, batches and the
    allocation-free entry point are refused before anything is launched."""
    from paper_2511_13905_amd import _native as N
    from paper_2511_13905_amd.api import project_noalloc
    p = I.many_rows(21, m=9, grid=(16, 8, 8))
    say("wide refusals", p.m)
    with pytest.raises(N.PgdtoError):
        ctx.project("coupled", dev(p.y.astype(np.float64)), dev(p.A.astype(np.float64)), p.b, p.lo, p.hi, p.C)
    res = torch.zeros(4096, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(N.PgdtoError) as e:
        project_noalloc("coupled", dev(p.y), dev(p.A), p.b, p.lo, p.hi, res, C=p.C, x=torch.empty_like(dev(p.y)))
    assert e.value.status == N.ERR_SCRATCH
    with pytest.raises(N.PgdtoError):
        rho = dev(p.y)
        ctx.pgd_step("coupled", dev(p.A), rho, rho, dev(p.y), dev(p.y), torch.zeros_like(rho), np.zeros(p.m),
                     np.ones(p.m), 3, p.lo, p.hi)
