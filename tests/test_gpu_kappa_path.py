"""GPU tests of pgdto_kappa_path (Appendix A.2, the remark on choosing C:
for an infeasible subproblem the penalty trades constraint violation against
the distance the projection moves the point).  Each point of the GPU path
(warm-started from the previous one) is held to the oracle's independent
solve at the same C; the path must show the penalty method's monotonicity.
Every case prints its name first."""
import math

import numpy as np
import pytest

import oracle
from oracle import projection as P
from paper_2511_13905_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print("[case]", *a, flush=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2511_13905_amd.api import Context
    c = Context(0)
    yield c
    c.close()


def compare(p, gpu_pts, orc_pts, x_last):
    rows = p.dense_rows() if p.kind == "independent" else np.atleast_2d(p.A.astype(np.float64))
    sig = P.row_scale(rows, p.lo, p.hi)
    for g, o in zip(gpu_pts, orc_pts):
        assert g["kappa"] == pytest.approx(o["kappa"], rel=1e-12)
        assert abs(g["dist"] - o["dist"]) <= 1e-5 * o["dist"] + 1e-12, (g["C"], g["dist"], o["dist"])
        for j in range(p.m):
            assert abs(g["violation"][j] - o["violation"][j]) <= 1e-6 * sig[j], (g["C"], j)
            assert abs(g["lam"][j] - o["lam"][j]) <= 1e-6 * abs(o["lam"][j]) + 1e-300, (g["C"], j)
    # the last point's x is in x_last
    np.testing.assert_allclose(x_last.cpu().numpy().astype(np.float64), orc_pts[-1]["result"].x,
                               rtol=1e-5, atol=0)
    # violation norm down, distance up, as C grows
    vn = [math.sqrt(sum(v * v for v in g["violation"])) for g in gpu_pts]
    for a, b in zip(vn, vn[1:]):
        assert b <= a * (1 + 1e-9) + 1e-12
    for a, b in zip(gpu_pts, gpu_pts[1:]):
        assert b["dist"] >= a["dist"] * (1 - 1e-9)


@pytest.mark.parametrize("seed", [1, 3])
def test_kappa_path_coupled_infeasible(ctx, seed):
    """Odd seeds of the volume + centre-of-mass case are infeasible on the box."""
    p = I.volume_com(seed, grid=(48, 24, 24))
    Cs = [1e4, 1e6, 1e8, 1e10, 1e12]
    say("kappa path coupled", seed, p.n, Cs)
    y, A = dev(p.y), dev(p.A)
    x, pts = ctx.kappa_path(p.kind, y, A, p.b, p.lo, p.hi, Cs, tau=1e-4)
    torch.cuda.synchronize()
    ref = oracle.kappa_path(p.kind, p.y, p.A, p.b, p.lo, p.hi, Cs, tau=1e-4)
    compare(p, pts, ref, x)
    for g in pts:
        assert g["violation_over_tau"] == pytest.approx(g["max_violation"] / 1e-4, rel=1e-12)
        assert g["outcome"] in ("converged", "infeasible")


def test_kappa_path_single_row_and_auto(ctx):
    """An infeasible single row (saturated point at every C) and the automatic
    penalty (C < 0, tau = -C) in the same path."""
    rng = np.random.default_rng(31)
    n = 200_000
    y = rng.uniform(-0.5, 1.5, n).astype(np.float32)
    a = rng.uniform(0.1, 1.0, n).astype(np.float32)
    lo, hi = I.LO, I.HI
    b = np.array([P.fsum(a.astype(np.float64) * lo) - 5.0])
    p = I.Problem("single", y, a.reshape(1, n), b)
    Cs = [1e3, 1e6, -1e-3, 1e9]
    say("kappa path single", n, Cs)
    x, pts = ctx.kappa_path(p.kind, dev(p.y), dev(p.A), p.b, p.lo, p.hi, Cs)
    torch.cuda.synchronize()
    ref = oracle.kappa_path(p.kind, p.y, p.A, p.b, p.lo, p.hi, Cs)
    sig = P.row_scale(np.atleast_2d(p.A.astype(np.float64)), lo, hi)[0]
    for g, o in zip(pts, ref):
        assert g["kappa"] == pytest.approx(o["kappa"], rel=1e-6)      # auto: breakpoint from a refined reciprocal
        # the GPU measures x as stored (float32 lo = 1e-3 rounds up by 4.7e-11
        # per element): the residual bar of the parity tests, 1e-6 sigma
        assert abs(g["max_violation"] - o["max_violation"]) <= 1e-6 * sig
        assert g["dist"] == pytest.approx(o["dist"], rel=1e-6)
        assert g["lam"][0] == pytest.approx(o["lam"][0], rel=1e-6)


def test_kappa_path_warm_starts_save_passes(ctx):
    """Continuation: a point started from its neighbour's multipliers takes
    no more passes than the same point solved cold."""
    p = I.volume_com(5, grid=(48, 24, 24))
    Cs = [1e10, 2e10, 4e10]
    say("kappa path warm", p.n, Cs)
    y, A = dev(p.y), dev(p.A)
    _, pts = ctx.kappa_path(p.kind, y, A, p.b, p.lo, p.hi, Cs)
    for g in pts[1:]:
        _, cold = ctx.project(p.kind, y, A, p.b, p.lo, p.hi, g["C"])
        assert g["passes"] <= cold["passes"], (g["C"], g["passes"], cold["passes"])
