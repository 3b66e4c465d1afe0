"""Algorithms 1 and 2 of the paper, as printed, in float64.

TEST INFRASTRUCTURE ONLY.  These follow the paper's steps in its own notation
(dual variable y <= 0, delta(y) = clip(sum_j y_j grad g_j, l - rho~, u - rho~))
and exist to report iteration counts and which branch of Algorithm 2 was
taken.  They are not a parity target: their stopping rules are the paper's
absolute tolerances, so they agree with ``projection.project`` only to within
those tolerances (checked in tests/test_oracle_literal.py).  Iteration counts
are "parity unpinned": reported, never compared with the GPU.

Readings where the printed algorithm is silent or cannot run as written:
  * elements with a zero gradient entry are left out of the bracket minimum
    (the printed quotient divides by zero there); the bracket end is clamped
    to y_l <= 0;
  * the bisection also stops when the midpoint equals an end point or after
    ``max_iter`` halvings, because an absolute tol_B below the float64 spacing
    of y_l never terminates;
  * the line search halves gamma from 1 (the paper asks for the largest
    gamma in (0, 1] satisfying both conditions, found by a binary-search
    scheme) and falls back to the largest Armijo gamma if none passes both;
  * after each Newton step y is clamped to y <= 0 (the printed Phi vanishes
    whenever h_j = 0, whatever the sign of y_j).
"""
from __future__ import annotations

import math

import numpy as np


def _fsum(v):
    return math.fsum(np.asarray(v, dtype=np.float64).ravel().tolist())


def _x_of(rho, A, yv, lo, hi):
    """rho~ + delta(y): the box clip of rho~ + sum_j y_j a_j (eq. delta_y)."""
    s = rho.copy()
    for j in range(A.shape[0]):
        if yv[j] != 0.0:
            s = s + yv[j] * A[j]
    return np.minimum(np.maximum(s, lo), hi), s


def alg1_bisection(rho, a, b, lo, hi, tol_b=1e-8, max_iter=200, kappa=0.0):
    """Algorithm 1 (single-constraint binary search).  Returns (y*, iterations).

    The feasibility test of Alg. 1 compares a.(rho~ + delta) with b (that is,
    (delta - alpha grad f)^T grad g - G + g > 0 with b = G - g + a.rho_t).
    ``kappa`` > 0 adds the regularization term of eq. (h) (used by Stage 1 of
    Algorithm 2 in its regularized reading); kappa = 0 is Alg. 1 as printed."""
    rho = np.asarray(rho, dtype=np.float64)
    a = np.asarray(a, dtype=np.float64)

    def viol(yv):
        x = np.minimum(np.maximum(rho + yv * a, lo), hi)
        return _fsum(a * x) - b + kappa * yv

    if viol(0.0) <= 0.0:
        return 0.0, 0
    nz = a != 0.0
    y_l = float(np.min(np.minimum((lo - rho[nz]) / a[nz], (hi - rho[nz]) / a[nz]))) if nz.any() else 0.0
    y_l = min(y_l, 0.0)
    if kappa > 0.0 and viol(y_l) > 0.0:
        # the regularized root lies past the last breakpoint (linear piece of slope kappa)
        return y_l - viol(y_l) / kappa, 0
    y_u = 0.0
    y_m = 0.5 * (y_u + y_l)
    it = 0
    while abs(y_u - y_l) > tol_b and it < max_iter:
        if viol(y_m) > 0.0:
            y_u = y_m
        else:
            y_l = y_m
        new = 0.5 * (y_u + y_l)
        it += 1
        if new == y_m or new == y_u or new == y_l:
            y_m = new
            break
        y_m = new
    return y_m, it


def alg2_newton(rho, A, b, lo, hi, C=1e12, tol_b=1e-8, tol_n=1e-6, maxiter=50,
                c1=1e-4, c2=0.9, max_halvings=30, stage1_kappa=True):
    """Algorithm 2 (Stage 1: single-active candidates; Stage 2: semismooth
    Newton on Phi with a line search on M = 1/2 ||Phi||^2).

    Returns a dict: y (paper sign), branch ("stage1" or "newton"), newton
    iterations, line-search trials, and the stage-1 candidate index."""
    rho = np.asarray(rho, dtype=np.float64)
    A = np.atleast_2d(np.asarray(A, dtype=np.float64))
    b = np.asarray(b, dtype=np.float64)
    m = A.shape[0]
    kappa = 2.0 / C

    def h_of(yv):
        x, s = _x_of(rho, A, yv, lo, hi)
        return np.array([_fsum(A[j] * x) - b[j] + kappa * yv[j] for j in range(m)]), s

    # Stage 1: one bisection per row, candidate j has only y_j nonzero
    y_trial = np.zeros(m)
    for j in range(m):
        yj, _ = alg1_bisection(rho, A[j], b[j], lo, hi, tol_b, kappa=kappa if stage1_kappa else 0.0)
        y_trial[j] = yj
        cand = np.zeros(m)
        cand[j] = yj
        x, _ = _x_of(rho, A, cand, lo, hi)
        feasible = all(_fsum(A[k] * x) - b[k] <= tol_n for k in range(m))
        if feasible:
            return {"y": cand, "branch": "stage1", "candidate": j, "newton": 0, "ls": 0}

    def phi_and_jac(yv):
        h, s = h_of(yv)
        act = h > 0.0
        phi = np.maximum(h, 0.0) + np.sign(np.maximum(-h, 0.0)) * yv
        chi = ((s >= lo) & (s <= hi)).astype(np.float64)
        Jh = (A * chi) @ A.T + kappa * np.eye(m)
        D = np.diag(act.astype(np.float64))
        Jphi = D @ Jh + np.eye(m) - D
        return phi, Jphi

    yv = y_trial.copy()
    phi, Jphi = phi_and_jac(yv)
    k = 0
    ls_total = 0
    while np.max(np.abs(phi)) > tol_n and k < maxiter:
        delta = np.linalg.solve(Jphi, phi)
        M0 = 0.5 * float(np.dot(phi, phi))
        slope = float(np.dot(phi, phi))            # grad M^T Delta = ||Phi||^2
        gamma = 1.0
        best = None
        accepted = None
        for _ in range(max_halvings + 1):
            cand = np.minimum(yv - gamma * delta, 0.0)
            ph, Jp = phi_and_jac(cand)
            ls_total += 1
            armijo = 0.5 * float(np.dot(ph, ph)) <= M0 - c1 * gamma * slope
            curv = float(np.dot(Jp.T @ ph, delta)) <= c2 * slope
            if armijo and best is None:
                best = (cand, ph, Jp)
            if armijo and curv:
                accepted = (cand, ph, Jp)
                break
            gamma *= 0.5
        if accepted is None:
            accepted = best if best is not None else (cand, ph, Jp)
        yv, phi, Jphi = accepted
        k += 1
    return {"y": yv, "branch": "newton", "candidate": -1, "newton": k, "ls": ls_total}
