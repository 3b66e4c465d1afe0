"""One step of Algorithm 3 (full PGD loop body) around the projection, float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Step size: Sec. 3.4.1 (eq. alpha, eq. final_alpha) with the first-step and
fallback rule of Alg. 3 and Sec. 3.4.3 (alpha = min(alpha_max, alpha_fallback /
||grad f||_inf)).  Direction: Sec. 3.4.2, eq. (CG), Polak-Ribiere with restart
(beta clipped at 0); Fletcher-Reeves and plain gradient are options.
Constraint right-hand side: the linearized row g_j + a_j.(x - rho_t) <= G_j,
i.e. b_j = G_j - g_j + a_j.rho_t (the paper's G-hat assumes rho~ = rho_t -
alpha grad f; Alg. 3 steps along omega alpha d_t instead, and this form is
identical to the paper's when omega = 1 and d = -grad f).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .projection import fsum, project


@dataclass
class PgdParams:
    """Defaults from Sec. 3.5 (C, alpha_max, tol_B, tol_N), Sec. 3.3 (alpha
    fallback 0.2), Sec. 3.4.1 (eps_alpha 1e-6) and Sec. 3.4.3 (t_warmup 50,
    omega 1)."""
    alpha_max: float = 1e2
    alpha_fallback: float = 0.2
    eps_alpha: float = 1e-6
    t_warmup: int = 50
    omega: float = 1.0
    tol_n: float = 1e-6       # constraint-violation threshold of the fallback rule
    tol: float = 1e-4         # stop test ||rho_{t+1} - rho_t|| / ||rho_{t+1}|| <= tol
    cg_rule: str = "pr+"      # "pr+" (paper), "fr", "none"


def step_size(rho, rho_prev, grad, grad_prev, g, G, t, p: PgdParams):
    """alpha_t of Alg. 3: the fallback step at t = 0 or (after warm-up) when the
    constraint violation ||max(g - G, 0)||_inf exceeds tol_N; otherwise the
    spectral step of eq. (final_alpha).  Returns (alpha, used_fallback)."""
    gmax = float(np.max(np.abs(grad))) if grad.size else 0.0
    fallback = (p.alpha_max if gmax == 0.0 else min(p.alpha_max, p.alpha_fallback / gmax))
    viol = float(np.max(np.maximum(np.asarray(g) - np.asarray(G), 0.0), initial=0.0))
    if t == 0 or (t >= p.t_warmup and viol > p.tol_n):
        return fallback, True
    s = rho - rho_prev
    yv = grad - grad_prev
    ss = fsum(s * s)
    yy = fsum(yv * yv)
    sy = fsum(s * yv)
    if yy == 0.0:
        return fallback, True
    lip = math.sqrt(ss) / math.sqrt(yy)                  # eq. (alpha)
    if sy > p.eps_alpha:
        return min(ss / sy, 2.0 * lip, p.alpha_max), False
    return min(lip, p.alpha_max), False


def cg_beta(grad, grad_prev, t, rule="pr+"):
    """beta_t of eq. (CG): max(grad_t.(grad_t - grad_{t-1}) / ||grad_{t-1}||^2, 0)
    (Polak-Ribiere with restart); d_0 = -grad f_0 means beta = 0 at t = 0."""
    if t == 0 or rule == "none":
        return 0.0
    gg_prev = fsum(grad_prev * grad_prev)
    if gg_prev == 0.0:
        return 0.0
    if rule == "fr":
        return fsum(grad * grad) / gg_prev
    return max(fsum(grad * (grad - grad_prev)) / gg_prev, 0.0)


def pgd_step(kind, rho, rho_prev, grad, grad_prev, d_prev, A, g, G, t, lo, hi,
             C=math.inf, offsets=None, p: PgdParams | None = None, stream_dtype=None):
    """One iteration body of Alg. 3: alpha_t, beta_t, d_t = -grad + beta d_{t-1},
    rho~ = rho_t + omega alpha_t d_t, rho_{t+1} = projection of rho~, and the
    relative-change stop test.  All arithmetic in float64.

    ``stream_dtype``: the precision in which rho~ and rho_{t+1} are stored
    (the paper does not fix one).  With float32 streams rho~ is a float32
    array like any other input of the projection, so it is rounded once here,
    and the stop test is taken on rho_{t+1} rounded to float32, the iterate
    the next step starts from; everything else stays float64."""
    p = p or PgdParams()
    f64 = lambda v: np.asarray(v, dtype=np.float64)
    rho, rho_prev, grad, grad_prev, d_prev = map(f64, (rho, rho_prev, grad, grad_prev, d_prev))
    g = f64(g).reshape(-1)
    G = f64(G).reshape(-1)
    alpha, used_fb = step_size(rho, rho_prev, grad, grad_prev, g, G, t, p)
    beta = cg_beta(grad, grad_prev, t, p.cg_rule)
    d = -grad + beta * d_prev
    rho_t = rho + p.omega * alpha * d
    if stream_dtype is not None and np.dtype(stream_dtype) != np.float64:
        rho_t = rho_t.astype(stream_dtype).astype(np.float64)
    if kind == "independent":
        c = f64(A).reshape(-1)
        arho = np.array([fsum(c[int(offsets[j]):int(offsets[j + 1])] * rho[int(offsets[j]):int(offsets[j + 1])])
                         for j in range(g.size)])
    else:
        Ad = np.atleast_2d(f64(A))
        arho = np.array([fsum(Ad[j] * rho) for j in range(Ad.shape[0])])
    b = G - g + arho
    res = project(kind, rho_t, A, b, lo, hi, C, offsets)
    # the stop test measures rho_{t+1} as it is stored: the next iterate is the
    # stored array, so with float32 streams x is rounded once before the test
    x_st = res.x
    if stream_dtype is not None and np.dtype(stream_dtype) != np.float64:
        x_st = res.x.astype(stream_dtype).astype(np.float64)
    diff = x_st - rho
    num = math.sqrt(fsum(diff * diff))
    den = math.sqrt(fsum(x_st * x_st))
    rel = num / den if den > 0.0 else math.inf
    return {"alpha": alpha, "beta": beta, "used_fallback": used_fb, "d": d, "rho_tilde": rho_t,
            "b": b, "proj": res, "x": res.x, "x_stored": x_st, "rel_change": rel, "converged": rel <= p.tol}
