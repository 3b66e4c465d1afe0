"""Parity checks of a GPU projection against the CPU oracle (shared by GPU tests).

Bar (from the build's stated tolerances):
  x            elementwise |x_gpu - x_orc| <= 1e-5 |x_orc| (box lower bound > 0),
               or <= 1e-5 max(1, |x_orc|) absolute when the box reaches 0;
  residual     |r_gpu - r_orc| <= 1e-6 |b_j| (1e-6 sigma_j when b_j is zero up to
               rounding, |b_j| <= 1e-9 sigma_j), plus the rounding of the stored x
               (the GPU residual is a_j.x with x as stored, the oracle's x is
               float64): half an ulp of the stream dtype at max(|lo|, |hi|) per
               element, 2^-24 sigma_j for float32 x;
  free set     identical for every element farther than 1e-6 from a bound
               (z from the oracle's float64 multiplier);
  multiplier   reported, compared per call site (it is not unique at kappa = 0
               on a plateau and ill-conditioned along null directions of A).
"""
import numpy as np

from oracle import projection as P


def free_from_mask(mask_words, n):
    w = np.asarray(mask_words, dtype=np.uint32)
    bits = np.unpackbits(w.view(np.uint8), bitorder="little")
    return bits[:n].astype(bool)


def check(prob, x_gpu, res, ref, free_gpu=None, xtol=1e-5, rtol_resid=1e-6, band=1e-6):
    x = np.asarray(x_gpu, dtype=np.float64)
    lo, hi = prob.lo, prob.hi
    scale = np.abs(ref.x) if lo > 0 else np.maximum(1.0, np.abs(ref.x))
    xerr = float(np.max(np.abs(x - ref.x) / scale))
    assert xerr <= xtol, f"x mismatch {xerr:.3e}"
    A = prob.dense_rows() if prob.kind == "independent" else np.atleast_2d(prob.A.astype(np.float64))
    sig = P.row_scale(A, lo, hi)
    m = prob.m
    xround = 2.0 ** -24 if np.asarray(x_gpu).dtype == np.float32 else 2.0 ** -53
    for j in range(m):
        ref_r = ref.resid[j]
        # rows whose b is zero up to rounding (e.g. b = G - g + a.rho with g = a.rho) use sigma_j
        bj = abs(prob.b[j])
        tol = rtol_resid * (bj if bj > 1e-9 * sig[j] else sig[j]) + xround * sig[j]
        assert abs(res["resid"][j] - ref_r) <= tol, (j, res["resid"][j], ref_r, tol)
    z = ref.z
    far = np.minimum(np.abs(z - lo), np.abs(z - hi)) > band
    orc_free = (z >= lo) & (z <= hi)
    if free_gpu is None:
        xt = np.asarray(x_gpu)
        free_gpu = (xt != xt.dtype.type(lo)) & (xt != xt.dtype.type(hi))
    mism = int(np.count_nonzero((free_gpu != orc_free) & far))
    assert mism == 0, f"free-set mismatch on {mism} elements"
    return {"xerr": xerr, "n_far": int(far.sum())}
