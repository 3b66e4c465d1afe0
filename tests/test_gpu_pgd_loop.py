"""Algorithm 3 driven for many iterations through pgdto_pgd_step.

A synthetic L-smooth objective stands in for the finite-element compliance
(which is outside the projection path): f(rho) = 1/2 sum_i w_i (rho_i - c_i)^2
+ mu/2 sum over grid neighbours (rho_i - rho_k)^2 on a 2-D grid, with linear
constraints (so their linearization is exact).  Its gradient is evaluated on
the host in float64 and handed to the GPU as float32, like any gradient from
an outside solver.

Every iteration is checked against the float64 oracle's Algorithm 3 step on
the very same float32 inputs (step size, beta, direction, the projected point
and the stop test), so the parity bar applies per iteration; over the run the
objective must fall and the iterates stay feasible.  The run also crosses the
first step (fallback step size), the warm-up boundary and the PR+ restarts.
The warm variants start each projection from the previous step's multipliers
(pgdto_problem.lambda0) and also run the cold step on the same inputs: the
warm run may take no more passes in total than the cold one.
"""
import numpy as np
import pytest

import oracle
from oracle.pgd import PgdParams
from paper_2511_13905_amd import inputs as I

from parity import check

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2511_13905_amd.api import Context
    c = Context(0)
    yield c
    c.close()


def say(*a):
    print("[case]", *a, flush=True)


class Objective:
    def __init__(self, nx, ny, seed, mu=0.5):
        rng = np.random.default_rng(seed)
        self.nx, self.ny, self.mu = nx, ny, mu
        self.c = rng.uniform(-0.2, 1.2, nx * ny)
        self.w = rng.uniform(0.5, 1.5, nx * ny)

    def value(self, r):
        g = r.reshape(self.ny, self.nx)
        lap = np.sum(np.diff(g, axis=0) ** 2) + np.sum(np.diff(g, axis=1) ** 2)
        return 0.5 * np.sum(self.w * (r - self.c) ** 2) + 0.5 * self.mu * lap

    def grad(self, r):
        g = r.reshape(self.ny, self.nx)
        L = np.zeros_like(g)
        dx = np.diff(g, axis=1)
        dy = np.diff(g, axis=0)
        L[:, :-1] -= dx
        L[:, 1:] += dx
        L[:-1, :] -= dy
        L[1:, :] += dy
        return self.w * (r - self.c) + self.mu * L.reshape(-1)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


@pytest.mark.parametrize("kind,rule,steps,warm", [("single", "pr+", 70, False), ("single", "fr", 20, False),
                                                 ("coupled", "pr+", 60, False), ("single", "pr+", 70, True),
                                                 ("coupled", "pr+", 60, True)])
def test_pgd_loop(ctx, kind, rule, steps, warm):
    nx, ny = 128, 64
    n = nx * ny
    obj = Objective(nx, ny, seed=3)
    lo, hi = I.LO, I.HI
    if kind == "single":
        A = np.full((1, n), 1.0 / n)            # mean(rho) <= 0.4
        G = np.array([0.4])
        C = np.inf
    else:
        # volume <= 0.4 and a centre-of-mass band in x, as linear rows
        p = I.volume_com(0, grid=(nx, ny), vf=0.4)
        A = p.A.astype(np.float64)
        G = p.b.copy()
        C = p.C
    A32 = A.astype(np.float32)
    Ad = A32.astype(np.float64)
    hyper = PgdParams(cg_rule=rule)
    say("pgd loop", kind, rule, steps, n, "warm" if warm else "cold")
    rho = np.full(n, 0.4, dtype=np.float32)
    rho_prev = grad_prev = None
    d = torch.zeros(n, dtype=torch.float32, device="cuda:0")
    A_dev = dev(A32)
    fvals = []
    fallbacks = []
    lam_prev = None
    passes_warm = passes_cold = 0
    for t in range(steps):
        gr = obj.grad(rho.astype(np.float64)).astype(np.float32)
        g = Ad @ rho.astype(np.float64)                      # constraint values (exact for linear rows)
        d_prev = d.cpu().numpy()
        args = (dev(rho), dev(rho_prev) if rho_prev is not None else None,
                dev(gr), dev(grad_prev) if grad_prev is not None else None)
        if warm:
            dc = d.clone()
            _, outc = ctx.pgd_step(kind, A_dev, *args, dc, g, G, t, lo, hi, C=C, cg_rule=rule)
            passes_cold += outc["proj"]["passes"]
        x, out = ctx.pgd_step(kind, A_dev, *args, d, g, G, t, lo, hi, C=C, cg_rule=rule,
                              lam0=lam_prev if warm else None)
        torch.cuda.synchronize()
        passes_warm += out["proj"]["passes"]
        lam_prev = [max(0.0, v) for v in out["proj"]["lam"]]
        xs = x.cpu().numpy()
        ref = oracle.pgd_step(kind, rho, rho_prev if rho_prev is not None else rho, gr,
                              grad_prev if grad_prev is not None else gr, d_prev, A32, g, G, t, lo, hi,
                              C=C, p=hyper, stream_dtype=np.float32)
        assert out["used_fallback"] == ref["used_fallback"], t
        assert np.isclose(out["alpha"], ref["alpha"], rtol=1e-9, atol=0), (t, out["alpha"], ref["alpha"])
        # beta = max(g.(g - g_prev), 0) / |g_prev|^2 cancels near stagnation: absolute bar
        assert np.isclose(out["beta"], ref["beta"], rtol=1e-9, atol=1e-12), (t, out["beta"], ref["beta"])
        dn = d.cpu().numpy().astype(np.float64)
        assert np.allclose(dn, ref["d"], rtol=1e-6, atol=1e-6 * np.max(np.abs(ref["d"]))), t
        prob = I.Problem(kind=kind, y=ref["rho_tilde"], A=A32, b=ref["b"], lo=lo, hi=hi, C=C)
        check(prob, xs, out["proj"], ref["proj"])
        # the stop test is taken on rho_{t+1} as stored (float32) on both sides
        assert np.isclose(out["rel_change"], ref["rel_change"], rtol=1e-5, atol=0), \
            (t, out["rel_change"], ref["rel_change"])
        assert out["converged"] == ref["converged"], t
        fallbacks.append(out["used_fallback"])
        rho_prev, grad_prev, rho = rho, gr, xs
        fvals.append(obj.value(rho.astype(np.float64)))
    assert fallbacks[0] and not all(fallbacks[1:])
    # the start point is infeasible for the coupled rows: compare from the first feasible iterate on
    assert fvals[-1] <= fvals[0]
    if rule == "pr+":
        # PR+ restarts keep the run settled at its best value (FR need not be monotone)
        assert min(fvals) >= fvals[-1] - 1e-6 * abs(fvals[-1])
    viol = Ad @ rho.astype(np.float64) - G
    assert np.max(viol) <= 1e-5 * max(1.0, float(np.max(np.abs(G))))
    if warm:
        print("passes over the run: warm", passes_warm, "cold", passes_cold, flush=True)
        assert passes_warm <= passes_cold
