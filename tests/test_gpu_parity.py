"""GPU parity: the HIP projection (through the C ABI) against the CPU oracle.

Every case prints its name, seed and shape before touching the GPU.
"""
import math

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


def run(ctx, p, params=None, want_mask=True):
    y = dev(p.y)
    A = dev(p.A)
    mask = torch.zeros((p.n + 31) // 32, dtype=torch.int32, device="cuda:0") if want_mask else None
    x, r = ctx.project(p.kind, y, A, p.b, p.lo, p.hi, p.C, offsets=p.offsets, free_mask=mask, params=params)
    torch.cuda.synchronize()
    xm = x.cpu().numpy()
    fm = free_from_mask(mask.cpu().numpy().view(np.uint32), p.n) if want_mask else None
    return xm, r, fm


def orc(p):
    return oracle.project(p.kind, p.y, p.A, p.b, p.lo, p.hi, p.C, p.offsets)


# ------------------------------------------------------------------ single row

@pytest.mark.parametrize("seed", range(12))
def test_volume_2d_f64(ctx, seed):
    p = I.volume_2d(seed, vf=0.5)
    say("volume_2d f64", seed, p.n)
    x, r, fm = run(ctx, p)
    ref = orc(p)
    check(p, x, r, ref, fm)
    assert r["outcome"] == ref.outcome[0]
    if ref.outcome[0] == "inactive":
        np.testing.assert_array_equal(x, np.clip(p.y, p.lo, p.hi))
    else:
        assert r["lam"][0] == pytest.approx(ref.lam[0], rel=1e-9)


@pytest.mark.parametrize("n", [1, 3, 5, 1000, 4097, 65537, 200003])
def test_compliance_ragged_f32(ctx, n):
    p = I.compliance_3d(n % 7, n=n)
    say("compliance f32 ragged", n)
    x, r, fm = run(ctx, p)
    ref = orc(p)
    check(p, x, r, ref, fm)
    assert r["outcome"] == ref.outcome[0]
    assert r["lam"][0] == pytest.approx(ref.lam[0], rel=1e-9, abs=1e-12)


def test_compliance_full_size(ctx):
    p = I.compliance_3d(0)
    say("compliance f32 full", p.n)
    x, r, fm = run(ctx, p)
    ref = orc(p)
    info = check(p, x, r, ref, fm)
    assert r["lam"][0] == pytest.approx(ref.lam[0], rel=1e-9)
    assert r["passes"] <= 16
    print("passes", r["passes"], info, flush=True)


def test_compliance_f64(ctx):
    p = I.compliance_3d(5, n=300001, dtype=np.float64)
    say("compliance f64", p.n)
    x, r, fm = run(ctx, p)
    check(p, x, r, orc(p), fm)


# ------------------------------------------------------------------ independent blocks

@pytest.mark.parametrize("n_per", [1, 7, 30001, 131072])
def test_multimaterial(ctx, n_per):
    p = I.multi_material(n_per % 5, fields=4, n_per=n_per)
    say("multimaterial", n_per)
    x, r, fm = run(ctx, p)
    ref = orc(p)
    check(p, x, r, ref, fm)
    for j in range(4):
        assert r["row_outcome"][j] == ref.outcome[j]
        assert r["lam"][j] == pytest.approx(ref.lam[j], rel=1e-9, abs=1e-9)


def test_multimaterial_full_size(ctx):
    p = I.multi_material(0)
    say("multimaterial full", p.n)
    x, r, fm = run(ctx, p)
    ref = orc(p)
    check(p, x, r, ref, fm)


def test_many_uneven_blocks(ctx):
    """64 blocks (the maximum) of uneven, unaligned sizes; mixed active/inactive."""
    rng = np.random.default_rng(44)
    sizes = rng.integers(1, 9000, 64)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    n = int(off[-1])
    y = rng.uniform(-0.3, 1.3, n).astype(np.float32)
    c = (1.0 / np.repeat(sizes, sizes)).astype(np.float32)
    caps = rng.uniform(0.1, 0.8, 64)
    p = I.Problem("independent", y, c, caps, offsets=off)
    say("many blocks", n)
    x, r, fm = run(ctx, p)
    ref = orc(p)
    check(p, x, r, ref, fm)
    assert [o for o in r["row_outcome"]] == ref.outcome


# ------------------------------------------------------------------ coupled rows

@pytest.mark.parametrize("seed", range(6))
def test_volume_com_small(ctx, seed):
    p = I.volume_com(seed, grid=(32, 16, 16))
    say("volume_com small", seed, p.n)
    x, r, fm = run(ctx, p)
    ref = orc(p)
    check(p, x, r, ref, fm)
    print(r["path"], r["passes"], r["iters_newton"], flush=True)


@pytest.mark.parametrize("seed", [0, 1])
def test_volume_com_f64(ctx, seed):
    """The coupled kernel on float64 streams (feasible and infeasible seeds)."""
    p = I.volume_com(seed, grid=(48, 24, 24), dtype=np.float64)
    say("volume_com f64", seed, p.n)
    x, r, fm = run(ctx, p)
    assert x.dtype == np.float64
    check(p, x, r, orc(p), fm)


def test_volume_com_ragged_2d(ctx):
    """n = 2 * 37^2 = 2738 is not a multiple of the vector width: rows are padded."""
    p = I.volume_com(2, grid=(74, 37))
    say("volume_com 2d ragged", p.n)
    x, r, fm = run(ctx, p)
    check(p, x, r, orc(p), fm)


@pytest.mark.parametrize("seed", [0, 1])
def test_volume_com_full_size(ctx, seed):
    p = I.volume_com(seed)
    say("volume_com full", seed, p.n)
    x, r, fm = run(ctx, p)
    ref = orc(p)
    check(p, x, r, ref, fm)
    print("path", r["path"], "passes", r["passes"], "newton", r["iters_newton"], flush=True)


@pytest.mark.parametrize("m", [1, 2, 3, 4, 6, 8])
def test_coupled_row_counts(ctx, m):
    """Random coupled rows, planted so that about half are active."""
    rng = np.random.default_rng(100 + m)
    n = 6000
    y = rng.uniform(-0.2, 1.2, n).astype(np.float32)
    A = (rng.standard_normal((m, n)) / n).astype(np.float32)
    A64 = A.astype(np.float64)
    lam = np.where(np.arange(m) % 2 == 0, rng.uniform(1, 5, m) * n, 0.0)
    xs, _ = P.clip_map(y.astype(np.float64), A64, lam, I.LO, I.HI)
    b = A64 @ xs + np.where(lam > 0, 0.0, 1e-3)
    p = I.Problem("coupled", y, A, b, C=1e12)
    say("coupled m", m)
    x, r, fm = run(ctx, p)
    check(p, x, r, orc(p), fm)


def test_coupled_paper_ncp_and_no_stage1(ctx):
    p = I.volume_com(0, grid=(32, 16, 16))
    ref = orc(p)
    for params in ({"ncp": "paper"}, {"stage1": 0}, {"ncp": "paper", "stage1": 0}):
        say("coupled variant", params)
        x, r, fm = run(ctx, p, params=params)
        check(p, x, r, ref, fm)


# ------------------------------------------------------------------ edge cases

def test_bisect_rule(ctx):
    """The printed midpoint rule (Alg. 1) with a tight tol_B reaches the same x."""
    p = I.volume_2d(3, vf=0.4)
    x, r, fm = run(ctx, p, params={"search": "bisect"})
    check(p, x, r, orc(p), fm)
    assert r["iters_search"] >= 30
    q = I.compliance_3d(1, n=100000)
    x, r, fm = run(ctx, q, params={"search": "bisect", "tol_b": 1e-14})
    check(q, x, r, orc(q), fm)


@pytest.mark.parametrize("kind", ["single", "independent", "coupled", "coupled-infeasible"])
def test_automatic_penalty(ctx, kind):
    """C < 0 asks for Appendix A.2's penalty C = 2 bp / tau (tau = -C) from
    the largest breakpoint of the zero pass; the oracle takes the same C from
    its own exact breakpoints."""
    import dataclasses
    gen = {"single": lambda: I.compliance_3d(2, n=70001),
           "independent": lambda: I.multi_material(1, fields=4, n_per=20001),
           "coupled": lambda: I.volume_com(0, grid=(96, 48)),
           "coupled-infeasible": lambda: I.volume_com(1, grid=(64, 32))}[kind]
    p0 = gen()
    tau = 1e-6 * float(np.max(np.abs(p0.b)))
    p = dataclasses.replace(p0, C=-tau)
    say("automatic penalty", kind, p.n, tau)
    x, r, fm = run(ctx, p)
    C_or = oracle.auto_C(p.kind, p.y, p.A, p.lo, p.hi, tau, p.offsets)
    assert math.isfinite(C_or)
    assert r["kappa"] == pytest.approx(2.0 / C_or, rel=1e-12)
    ref = oracle.project(p.kind, p.y, p.A, p.b, p.lo, p.hi, C_or, p.offsets)
    check(dataclasses.replace(p0, C=C_or), x, r, ref, fm)
    if kind in ("single", "independent"):
        for j in range(p.m):
            assert r["resid"][j] <= tau * (1 + 1e-6) + 1e-6 * abs(p.b[j])


def _eq_case(case):
    if case.startswith("single"):
        p = I.compliance_3d(4, n=50001)
        if case == "single-raise":       # a.clip(y) below b: lam < 0 lifts the row to b
            ax = float(p.A[0].astype(np.float64) @ np.clip(p.y.astype(np.float64), p.lo, p.hi))
            p.b = np.array([ax + 0.3 * abs(ax)])
        return p, [True]
    if case == "independent":
        p = I.multi_material(2, fields=4, n_per=30001)
        p.b = p.b.copy()
        p.b[0] = 0.7                     # above the field's mean: lifted
        p.b[2] = 0.4
        return p, [True, False, True, False]
    p = I.volume_com(0, grid=(96, 48))
    p.b = p.b.copy()
    p.b[0] = 0.45 * float(np.sum(p.A[0]))   # volume held at 45%, above clip(y)'s
    return p, [True, False, False, False, False]


@pytest.mark.parametrize("case", ["single-lower", "single-raise", "independent", "coupled"])
def test_equality_rows(ctx, case):
    """Rows held at equality (Sec. 3.2): always active, multiplier of either
    sign.  The HIP path against the oracle's equality solve."""
    p, eq = _eq_case(case)
    say("equality rows", case, p.n, eq)
    y, A = dev(p.y), dev(p.A)
    mask = torch.zeros((p.n + 31) // 32, dtype=torch.int32, device="cuda:0")
    x, r = ctx.project(p.kind, y, A, p.b, p.lo, p.hi, p.C, offsets=p.offsets, free_mask=mask, eq=eq)
    torch.cuda.synchronize()
    fm = free_from_mask(mask.cpu().numpy().view(np.uint32), p.n)
    ref = oracle.project(p.kind, p.y, p.A, p.b, p.lo, p.hi, p.C, p.offsets, eq=eq)
    check(p, x.cpu().numpy(), r, ref, fm)
    for j, e in enumerate(eq):
        assert r["lam"][j] == pytest.approx(ref.lam[j], rel=1e-6, abs=1e-9 * max(1.0, abs(ref.lam[j]))), j
        if e:
            sig = P.row_scale(np.atleast_2d(p.dense_rows() if p.kind == "independent" else p.A), p.lo, p.hi)[j]
            assert abs(r["resid"][j] - r["slack"][j]) <= 1e-6 * max(abs(p.b[j]), 1e-9 * sig)
    if case in ("single-raise", "independent", "coupled"):
        assert r["lam"][0] < 0.0



def _warm_run(ctx, p, lam0, eq=None):
    y, A = dev(p.y), dev(p.A)
    mask = torch.zeros((p.n + 31) // 32, dtype=torch.int32, device="cuda:0")
    x, r = ctx.project(p.kind, y, A, p.b, p.lo, p.hi, p.C, offsets=p.offsets, free_mask=mask, eq=eq, lam0=lam0)
    torch.cuda.synchronize()
    return x.cpu().numpy(), r, free_from_mask(mask.cpu().numpy().view(np.uint32), p.n)


WARM_CASES = {
    "single": lambda: I.compliance_3d(0),
    "independent": lambda: I.multi_material(2, fields=4, n_per=131072),
    "coupled": lambda: I.volume_com(0, grid=(48, 24, 24)),
    "coupled-infeasible": lambda: I.volume_com(1, grid=(48, 24, 24)),
}


@pytest.mark.parametrize("case", list(WARM_CASES))
@pytest.mark.parametrize("factor", [1.0, 0.97, 1.05])
def test_warm_start(ctx, case, factor):
    """pgdto_problem.lambda0: a warm start changes the search path, not the
    projection.  Started from the oracle's multipliers (scaled), the HIP path
    still matches the oracle; from the exact ones a 1-D search ends in one
    pass (zero pass, one search pass, final pass)."""
    p = WARM_CASES[case]()
    ref = orc(p)
    lam0 = [max(0.0, float(v) * factor) for v in ref.lam]
    say("warm start", case, factor, p.n, lam0)
    xc, rc, _ = run(ctx, p)
    x, r, fm = _warm_run(ctx, p, lam0)
    check(p, x, r, ref, fm)
    print("cold passes", rc["passes"], "warm passes", r["passes"], "path", r["path"], flush=True)
    if p.kind != "coupled" and factor == 1.0:
        assert r["passes"] <= 3
    if p.kind == "coupled":
        assert r["path"] in (0, 3)


def test_warm_start_outside_bracket_is_ignored(ctx):
    """A lambda0 outside the 1-D bracket [0, largest breakpoint] leaves the
    search as it is: bitwise the cold result."""
    p = I.compliance_3d(3, n=1000003)
    say("warm start outside", p.n)
    xc, rc, fc = run(ctx, p)
    x, r, fm = _warm_run(ctx, p, [1e30])
    assert np.array_equal(x.view(np.uint32), xc.view(np.uint32))
    assert r["lam"] == rc["lam"] and r["passes"] == rc["passes"]
    assert np.array_equal(fm, fc)


@pytest.mark.parametrize("case", ["single-raise", "coupled"])
def test_warm_start_equality_rows(ctx, case):
    """Equality rows take a warm start of either sign."""
    p, eq = _eq_case(case)
    ref = oracle.project(p.kind, p.y, p.A, p.b, p.lo, p.hi, p.C, p.offsets, eq=eq)
    lam0 = [float(v) * 1.02 for v in ref.lam]
    say("warm start equality", case, p.n, lam0)
    x, r, fm = _warm_run(ctx, p, lam0, eq=eq)
    check(p, x, r, ref, fm)
    assert r["lam"][0] < 0.0
    assert r["lam"][0] == pytest.approx(ref.lam[0], rel=1e-6)


@pytest.mark.parametrize("warm", [False, True])
def test_graph_replay_matches_eager(ctx, warm):
    """One-instance launches captured in a HIP graph (two projections, masks
    included) and replayed three times, with eager launches on the same
    context between replays: every replay gives the bits of eager calls.
    warm: both start from the same lambda0 (1.01 x the oracle's multipliers),
    which the captured launch holds in its kernel argument."""
    from paper_2511_13905_amd.api import result_from_bytes, result_nbytes
    probs = [I.compliance_3d(6, n=100003), I.volume_com(1, grid=(64, 32))]
    lam0s = [[max(0.0, 1.01 * float(v)) for v in orc(p).lam] if warm else None for p in probs]
    say("graph replay", "warm" if warm else "cold", [p.n for p in probs])
    dev_in = [(dev(p.y), dev(p.A)) for p in probs]
    xs = [torch.empty(p.n, dtype=torch.float32, device="cuda:0") for p in probs]
    ms = [torch.zeros((p.n + 31) // 32, dtype=torch.int32, device="cuda:0") for p in probs]
    rs = [torch.zeros(result_nbytes(), dtype=torch.uint8, device="cuda:0") for _ in probs]

    def enqueue():
        for p, (y, A), x, m, r, l0 in zip(probs, dev_in, xs, ms, rs, lam0s):
            ctx.project_async(p.kind, y, A, p.b, p.lo, p.hi, r, C=p.C, offsets=p.offsets, x=x, free_mask=m,
                              lam0=l0)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        enqueue()                                    # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        enqueue()
    torch.cuda.synchronize()
    eager = []
    for p, (y, A), l0 in zip(probs, dev_in, lam0s):
        m = torch.zeros((p.n + 31) // 32, dtype=torch.int32, device="cuda:0")
        x, r = ctx.project(p.kind, y, A, p.b, p.lo, p.hi, p.C, offsets=p.offsets, free_mask=m, lam0=l0)
        torch.cuda.synchronize()
        eager.append((x.cpu().numpy(), m.cpu().numpy(), r))
    other = I.multi_material(5, fields=2, n_per=20011)
    for rep in range(3):
        for x, m in zip(xs, ms):
            x.fill_(-1.0)
            m.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for (xe, me, re_), x, m, r in zip(eager, xs, ms, rs):
            assert np.array_equal(x.cpu().numpy(), xe), rep
            assert np.array_equal(m.cpu().numpy(), me), rep
            rr = result_from_bytes(r)
            assert rr["lam"] == re_["lam"] and rr["passes"] == re_["passes"] and rr["error"] == 0, (rep, rr, re_)
        # an eager launch on the same context between replays
        ctx.project(other.kind, dev(other.y), dev(other.A), other.b, other.lo, other.hi, other.C,
                    offsets=other.offsets)
        torch.cuda.synchronize()


def test_graph_replay_pgd_step(ctx):
    """pgd_step_async captured once and replayed three times (d is updated in
    place, so every replay is the next step of the same sequence) gives the
    bits of three eager steps."""
    from paper_2511_13905_amd.api import result_from_bytes, result_nbytes
    st = I.pgd_compliance_3d(4, t=60, n=150001)
    say("graph replay pgd_step", st.rho.size)
    A, rho, rp, gr, gp = (dev(v) for v in (st.problem.A, st.rho, st.rho_prev, st.grad, st.grad_prev))
    # eager reference: three steps on one direction buffer
    d_e = dev(st.d_prev)
    eager = []
    for _ in range(3):
        x, out = ctx.pgd_step("single", A, rho, rp, gr, gp, d_e, st.g, st.G, st.t, I.LO, I.HI)
        torch.cuda.synchronize()
        eager.append((x.cpu().numpy(), d_e.cpu().numpy(), out))
    d_g = dev(st.d_prev)
    x_g = torch.empty_like(rho)
    res = torch.zeros(result_nbytes(pgd=True), dtype=torch.uint8, device="cuda:0")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):                     # warm-up outside the capture, on a scratch d
        d_w = dev(st.d_prev)
        ctx.pgd_step_async("single", A, rho, rp, gr, gp, d_w, st.g, st.G, st.t, I.LO, I.HI, res, x=x_g)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ctx.pgd_step_async("single", A, rho, rp, gr, gp, d_g, st.g, st.G, st.t, I.LO, I.HI, res, x=x_g)
    torch.cuda.synchronize()
    for k in range(3):
        g.replay()
        torch.cuda.synchronize()
        xe, de, oe = eager[k]
        assert np.array_equal(x_g.cpu().numpy(), xe), k
        assert np.array_equal(d_g.cpu().numpy(), de), k
        og = result_from_bytes(res, pgd=True)
        assert og["alpha"] == oe["alpha"] and og["proj"]["lam"] == oe["proj"]["lam"], k


def test_reduction_forms_give_the_same_bits(ctx):
    """The two forms of the per-pass grid reduction, every workgroup summing
    the tile partials itself (the default) and workgroup 0 summing them alone
    and publishing the totals with a go word (PGDTO_REDUCE_WG0=1; the form
    of launches above 256 workgroups), add the same partials in the same tile
    order: every kind gives the same bits either way."""
    import os
    from paper_2511_13905_amd.api import Context, result_from_bytes
    os.environ["PGDTO_REDUCE_WG0"] = "1"
    try:
        c0 = Context(0)
    finally:
        del os.environ["PGDTO_REDUCE_WG0"]
    p64 = I.compliance_3d(9, n=120001)
    p64.y = p64.y.astype(np.float64)
    p64.A = p64.A.astype(np.float64)
    probs = [I.compliance_3d(3, n=1_000_003), I.multi_material(5, fields=4, n_per=131_071),
             I.volume_com(0, grid=(96, 48, 24)), I.volume_com(1, grid=(96, 48, 24)), p64]
    say("reduction forms", [p.n for p in probs])
    try:
        for p in probs:
            outs = []
            for c in (c0, ctx):
                m = torch.zeros((p.n + 31) // 32, dtype=torch.int32, device="cuda:0")
                x, r = c.project(p.kind, dev(p.y), dev(p.A), p.b, p.lo, p.hi, p.C, offsets=p.offsets, free_mask=m)
                torch.cuda.synchronize()
                outs.append((x.cpu().numpy(), m.cpu().numpy(), r))
            (x0, m0, r0), (x1, m1, r1) = outs
            assert r0["error"] == 0 and r1["error"] == 0
            assert np.array_equal(x0, x1) and np.array_equal(m0, m1), p.kind
            assert r0["lam"] == r1["lam"] and r0["passes"] == r1["passes"] and r0["resid"] == r1["resid"], p.kind
        st = I.pgd_compliance_3d(4, t=60, n=400_001)
        pg = []
        for c in (c0, ctx):
            d = dev(st.d_prev)
            x, out = c.pgd_step("single", dev(st.problem.A), dev(st.rho), dev(st.rho_prev), dev(st.grad),
                                dev(st.grad_prev), d, st.g, st.G, st.t, I.LO, I.HI)
            torch.cuda.synchronize()
            pg.append((x.cpu().numpy(), d.cpu().numpy(), out))
        assert np.array_equal(pg[0][0], pg[1][0]) and np.array_equal(pg[0][1], pg[1][1])
        assert pg[0][2]["alpha"] == pg[1][2]["alpha"] and pg[0][2]["proj"]["lam"] == pg[1][2]["proj"]["lam"]
        assert pg[0][2]["rel_change"] == pg[1][2]["rel_change"]
    finally:
        c0.close()


def test_late_arrivals_give_the_same_bits(ctx):
    """An arrival door that closes at the first arrival (PGDTO_DOOR_WAIT=0)
    leaves most of the grid out: the participants solve every tile, late
    workgroups leave, the last of them reopens the door.  Several launches in
    a row of every kind give the bits of full-grid launches."""
    import os
    from paper_2511_13905_amd.api import Context
    os.environ["PGDTO_DOOR_WAIT"] = "0"
    try:
        c0 = Context(0)
    finally:
        del os.environ["PGDTO_DOOR_WAIT"]
    p64 = I.compliance_3d(8, n=90001)
    p64.y = p64.y.astype(np.float64)
    p64.A = p64.A.astype(np.float64)
    probs = [I.compliance_3d(7, n=200003), I.multi_material(6, fields=3, n_per=40011),
             I.volume_com(0, grid=(64, 32)), I.volume_com(1, grid=(48, 24)), p64]
    eqs = [None, [True, False, True], [True, False, False, False, False], None, None]
    say("late arrivals", [p.n for p in probs])
    st = I.pgd_compliance_3d(2, t=60, n=150001)
    try:
        for rep in range(2):
            for p, eq in zip(probs, eqs):
                outs = []
                for c in (c0, ctx):
                    m = torch.zeros((p.n + 31) // 32, dtype=torch.int32, device="cuda:0")
                    x, r = c.project(p.kind, dev(p.y), dev(p.A), p.b, p.lo, p.hi, p.C, offsets=p.offsets,
                                     free_mask=m, eq=(eq if rep == 1 else None))
                    torch.cuda.synchronize()
                    outs.append((x.cpu().numpy(), m.cpu().numpy(), r))
                (x0, m0, r0), (x1, m1, r1) = outs
                assert r0["error"] == 0 and r1["error"] == 0
                assert np.array_equal(x0, x1) and np.array_equal(m0, m1), (rep, p.kind)
                assert r0["lam"] == r1["lam"] and r0["passes"] == r1["passes"]
            pg = []
            for c in (c0, ctx):
                d = dev(st.d_prev)
                x, out = c.pgd_step("single", dev(st.problem.A), dev(st.rho), dev(st.rho_prev), dev(st.grad),
                                    dev(st.grad_prev), d, st.g, st.G, st.t, I.LO, I.HI)
                torch.cuda.synchronize()
                pg.append((x.cpu().numpy(), d.cpu().numpy(), out))
            assert np.array_equal(pg[0][0], pg[1][0]) and np.array_equal(pg[0][1], pg[1][1])
            assert pg[0][2]["alpha"] == pg[1][2]["alpha"] and pg[0][2]["proj"]["lam"] == pg[1][2]["proj"]["lam"]
        # Algorithm 3 on coupled rows and on independent blocks
        rng = np.random.default_rng(31)
        pc = I.volume_com(0, grid=(48, 24, 24))
        blocks = np.array([0, 9001, 18002, pc.n], dtype=np.int64)
        cases = [("coupled", pc.A, pc.b.copy(), pc.C, None),
                 ("independent", np.full(pc.n, 1.0 / 9001, dtype=np.float32), np.array([0.3, 0.25, 0.2]),
                  math.inf, blocks)]
        rho = np.clip(rng.uniform(0, 0.6, pc.n), I.LO, I.HI).astype(np.float32)
        grad = rng.standard_normal(pc.n).astype(np.float32)
        rho_prev = (rho - 0.01 * rng.standard_normal(pc.n)).astype(np.float32)
        grad_prev = (grad + 0.1 * rng.standard_normal(pc.n)).astype(np.float32)
        for kind, A, G, Cp, offs in cases:
            A64 = np.atleast_2d(A.astype(np.float64))
            if kind == "independent":
                g = np.array([float(A64[0, offs[j]:offs[j + 1]] @ rho[offs[j]:offs[j + 1]]) for j in range(3)])
            else:
                g = A64 @ rho.astype(np.float64)
            pg = []
            for c in (c0, ctx):
                d = dev(-grad_prev)
                x, out = c.pgd_step(kind, dev(A), dev(rho), dev(rho_prev), dev(grad), dev(grad_prev), d, g, G, 70,
                                    I.LO, I.HI, C=Cp, offsets=offs)
                torch.cuda.synchronize()
                pg.append((x.cpu().numpy(), d.cpu().numpy(), out))
            assert np.array_equal(pg[0][0], pg[1][0]) and np.array_equal(pg[0][1], pg[1][1]), kind
            assert pg[0][2]["proj"]["lam"] == pg[1][2]["proj"]["lam"], kind
    finally:
        c0.close()


def test_infeasible_single_row(ctx):
    rng = np.random.default_rng(12)
    n = 5000
    y = rng.uniform(-0.5, 1.5, n).astype(np.float32)
    a = rng.standard_normal(n).astype(np.float32)
    a64 = a.astype(np.float64)
    xmin = np.where(a64 > 0, I.LO, I.HI)
    b = float(a64 @ xmin) - 1.0
    p = I.Problem("single", y, a.reshape(1, n), np.array([b]))
    x, r, fm = run(ctx, p)
    ref = orc(p)
    assert r["outcome"] == "infeasible"
    check(p, x, r, ref, fm)


def test_nonfinite_input(ctx):
    p = I.compliance_3d(3, n=10000)
    p.y[17] = np.nan
    x, r, fm = run(ctx, p, want_mask=False)
    assert r["outcome"] == "nonfinite"


def test_inactive_bit_exact(ctx):
    p = I.compliance_3d(0, n=50000)
    p.b[:] = 1e9
    x, r, _ = run(ctx, p, want_mask=False)
    assert r["outcome"] == "inactive"
    np.testing.assert_array_equal(x, np.clip(p.y, np.float32(p.lo), np.float32(p.hi)).astype(np.float32)
                                  if False else np.clip(p.y.astype(np.float64), p.lo, p.hi).astype(np.float32))


def test_repeat_is_bitwise_identical(ctx):
    p = I.volume_com(0, grid=(48, 24, 24))
    x1, r1, _ = run(ctx, p, want_mask=False)
    x2, r2, _ = run(ctx, p, want_mask=False)
    np.testing.assert_array_equal(x1, x2)
    assert r1["lam"] == r2["lam"]


def test_invalid_arguments(ctx):
    from paper_2511_13905_amd import _native as N
    p = I.compliance_3d(0, n=4096)
    y, A = dev(p.y), dev(p.A)
    bad = [dict(lo=1.0, hi=0.5), dict(lo=float("nan"))]
    for kw in bad:
        args = dict(lo=p.lo, hi=p.hi)
        args.update(kw)
        with pytest.raises(N.PgdtoError) as e:
            ctx.project("single", y, A, p.b, args["lo"], args["hi"])
        assert e.value.status == N.ERR_ARG
    with pytest.raises(N.PgdtoError):
        ctx.project("single", y, A, p.b, p.lo, p.hi, x=y)          # x aliases y
    with pytest.raises(N.PgdtoError):
        ctx.project("single", y, A, [float("nan")], p.lo, p.hi)
    q = I.multi_material(0, n_per=1000)
    with pytest.raises(N.PgdtoError):
        ctx.project("independent", dev(q.y), dev(q.A), q.b, q.lo, q.hi, offsets=[0, 10, 5, 3000, 4000])
    with pytest.raises(N.PgdtoError):                                # misaligned y
        yy = torch.zeros(4097, dtype=torch.float32, device="cuda:0")[1:]
        ctx.project("single", yy, A, p.b, p.lo, p.hi)


# ------------------------------------------------------------------ Algorithm 3 step

@pytest.mark.parametrize("t,rule", [(60, "pr+"), (0, "pr+"), (60, "fr"), (10, "none")])
def test_pgd_step_single(ctx, t, rule):
    st = I.pgd_compliance_3d(1, t=t, n=200003)
    say("pgd_step", t, rule, st.rho.size)
    A = st.problem.A
    d = dev(st.d_prev)
    x, out = ctx.pgd_step("single", dev(A), dev(st.rho), dev(st.rho_prev), dev(st.grad), dev(st.grad_prev), d,
                          st.g, st.G, t, I.LO, I.HI, cg_rule=rule)
    torch.cuda.synchronize()
    ref = oracle.pgd_step("single", st.rho, st.rho_prev, st.grad, st.grad_prev, st.d_prev, A, st.g, st.G, t,
                          I.LO, I.HI, p=oracle.PgdParams(cg_rule=rule), stream_dtype=np.float32)
    assert out["alpha"] == pytest.approx(ref["alpha"], rel=1e-12)
    assert out["beta"] == pytest.approx(ref["beta"], rel=1e-9, abs=1e-15)
    assert out["used_fallback"] == ref["used_fallback"]
    np.testing.assert_allclose(d.cpu().numpy(), ref["d"], rtol=1e-6, atol=1e-7)
    prob = I.Problem("single", ref["rho_tilde"], A, ref["b"])
    check(prob, x.cpu().numpy(), out["proj"], ref["proj"])
    assert out["rel_change"] == pytest.approx(ref["rel_change"], rel=1e-5)


@pytest.mark.parametrize("t", [0, 70])
def test_pgd_step_independent(ctx, t):
    """Algorithm 3 on independent blocks (three material fields, one volume
    cap each): b_j = G_j - g_j + a_j.rho_t per block."""
    rng = np.random.default_rng(9 + t)
    n_per, m = 40011, 3
    n = n_per * m
    offsets = np.arange(m + 1, dtype=np.int64) * n_per
    A = np.full(n, 1.0 / n_per, dtype=np.float32)
    rho = np.clip(rng.uniform(0, 0.6, n), I.LO, I.HI).astype(np.float32)
    grad = rng.standard_normal(n).astype(np.float32)
    rho_prev = (rho - 0.01 * rng.standard_normal(n)).astype(np.float32)
    grad_prev = (grad + 0.1 * rng.standard_normal(n)).astype(np.float32)
    d_prev = (-grad_prev).astype(np.float32)
    A64 = A.astype(np.float64)
    g = np.array([float(A64[offsets[j]:offsets[j + 1]] @ rho[offsets[j]:offsets[j + 1]].astype(np.float64))
                  for j in range(m)])
    G = np.array([0.25, 0.3, 0.2])
    say("pgd_step independent", t, n)
    d = dev(d_prev)
    x, out = ctx.pgd_step("independent", dev(A), dev(rho), dev(rho_prev), dev(grad), dev(grad_prev), d, g, G, t,
                          I.LO, I.HI, offsets=offsets)
    torch.cuda.synchronize()
    ref = oracle.pgd_step("independent", rho, rho_prev, grad, grad_prev, d_prev, A, g, G, t, I.LO, I.HI,
                          offsets=offsets, stream_dtype=np.float32)
    assert out["alpha"] == pytest.approx(ref["alpha"], rel=1e-12)
    assert out["used_fallback"] == ref["used_fallback"]
    np.testing.assert_allclose(d.cpu().numpy(), ref["d"], rtol=1e-6, atol=1e-7)
    prob = I.Problem("independent", ref["rho_tilde"], A, ref["b"], offsets=offsets)
    check(prob, x.cpu().numpy(), out["proj"], ref["proj"])
    assert out["rel_change"] == pytest.approx(ref["rel_change"], rel=1e-5)


def test_pgd_step_coupled(ctx):
    p = I.volume_com(0, grid=(32, 16, 16))
    rng = np.random.default_rng(5)
    n = p.n
    rho = np.clip(rng.uniform(0, 1, n), I.LO, I.HI).astype(np.float32)
    grad = rng.standard_normal(n).astype(np.float32)
    rho_prev = (rho - 0.01 * rng.standard_normal(n)).astype(np.float32)
    grad_prev = (grad + 0.1 * rng.standard_normal(n)).astype(np.float32)
    d_prev = (-grad_prev).astype(np.float32)
    A64 = p.A.astype(np.float64)
    g = A64 @ rho.astype(np.float64)
    G = p.b.copy()
    d = dev(d_prev)
    x, out = ctx.pgd_step("coupled", dev(p.A), dev(rho), dev(rho_prev), dev(grad), dev(grad_prev), d, g, G, 70,
                          I.LO, I.HI, C=p.C)
    ref = oracle.pgd_step("coupled", rho, rho_prev, grad, grad_prev, d_prev, p.A, g, G, 70, I.LO, I.HI, C=p.C,
                          stream_dtype=np.float32)
    assert out["alpha"] == pytest.approx(ref["alpha"], rel=1e-12)
    prob = I.Problem("coupled", ref["rho_tilde"], p.A, ref["b"], C=p.C)
    check(prob, x.cpu().numpy(), out["proj"], ref["proj"])
