"""CPU float64 oracle for the PGD-TO projection hot path (arXiv 2511.13905).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
statement of what the projection computes, written from the paper's
definitions (Theorems 1 and 2, Appendix A).  Only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import
it.  It shares no code with the HIP library and never imports it.

Contents
  projection.exact_single    exact 1-row projection (Appendix A.1, eq. Gamma),
                              breakpoint search; kappa >= 0
  projection.project         dispatcher: single / independent / coupled
  projection.coupled          regularized multi-row projection (Appendix A.2):
                              dual maximization, active-pattern polish, KKT check
  projection.kkt_certificate  KKT residuals of eq. (rkkt1)-(rkkt11)
  projection.brute_force      enumeration of element states and active rows
  projection.auto_C           the penalty bounding constraint violation by tau
                              (Appendix A.2), from the largest breakpoint
  projection.kappa_path       the projection along a list of penalties C
                              (Appendix A.2: violation against distance)
  literal.alg1_bisection      Algorithm 1 as printed (float64), for iteration counts
  literal.alg2_newton         Algorithm 2 (Stage 1 + semismooth Newton), float64
  pgd.pgd_step                one step of Algorithm 3 around the projection

Parity pins for every function are in ``tests/test_oracle_*.py``.  The only
quantities left unpinned are the literal algorithms' iteration counts
("parity unpinned": they are reported, never compared).
"""
from .projection import (clip_map, h_map, exact_single, project, coupled,
                         kkt_certificate, brute_force, row_scale, OracleResult,
                         largest_breakpoint, auto_C, kappa_path)
from .pgd import pgd_step, step_size, cg_beta, PgdParams
from . import literal

__all__ = ["clip_map", "h_map", "exact_single", "project", "coupled", "kkt_certificate",
           "brute_force", "row_scale", "OracleResult", "largest_breakpoint", "auto_C", "kappa_path", "pgd_step", "step_size", "cg_beta",
           "PgdParams", "literal"]
