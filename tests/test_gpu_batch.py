"""Serving (pgdto_batch) on the GPU: the persistent multi-slot executor and the
plain path against single-launch projections and the CPU oracle.

Bitwise agreement with pgdto_project follows from the tile-ordered
reductions (the result does not depend on how many workgroups solve an
instance).  Every case prints its name before touching the GPU.
"""
import time

import numpy as np
import pytest

import oracle
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


def mixed_requests(seed, count, n_lo=4096, n_hi=120000):
    """Small requests of the served mix (sizes the oracle checks quickly)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(round(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi)))))
        kind = I.SERVE_KINDS[i % 3]
        out.append(I.serve_request(int(rng.integers(0, 2**31 - 1)), n, kind))
    return out


def stage(reqs, mask=True):
    """Device inputs of every request, written before any submit: the
    executor starts on a request as soon as it is published, in no stream
    order.  The free mask is deliberately not cleared (the executor does it)."""
    from paper_2511_13905_amd.api import aligned_rows
    out = []
    for p in reqs:
        fm = torch.full(((p.n + 31) // 32,), -1, dtype=torch.int32, device="cuda:0") if mask else None
        A = dev(p.A)
        if p.kind != "independent":
            A = aligned_rows(A)
        out.append((dev(p.y), A, fm))
    torch.cuda.synchronize()
    return out


def submit(B, p, staged):
    y, A, fm = staged
    t = B.submit(p.kind, y, A, p.b, p.lo, p.hi, p.C, offsets=p.offsets, free_mask=fm)
    return t, fm


def collect(B, t, fm, n):
    x = B.x_of(t)
    st, r, times = B.wait(t)
    torch.cuda.synchronize()
    mask = free_from_mask(fm.cpu().numpy().view(np.uint32), n) if fm is not None else None
    return st, r, x.cpu().numpy(), mask, times


def single(ctx, p):
    y, A = dev(p.y), dev(p.A)
    fm = torch.zeros((p.n + 31) // 32, dtype=torch.int32, device="cuda:0")
    x, r = ctx.project(p.kind, y, A, p.b, p.lo, p.hi, p.C, offsets=p.offsets, free_mask=fm)
    torch.cuda.synchronize()
    return x.cpu().numpy(), r, free_from_mask(fm.cpu().numpy().view(np.uint32), p.n)


def test_server_shape(ctx):
    from paper_2511_13905_amd.api import Batch
    say("server shape")
    B = Batch(ctx, max_slots=4)
    s, w = B.shape()
    B.close()
    assert s == 4 and w >= 1
    B = Batch(ctx, max_slots=1)
    assert B.shape() == (0, 0)
    B.close()


def test_batch_autotune_picks_fastest_shape(ctx):
    from paper_2511_13905_amd.api import TUNE_SLOTS, Batch, aligned_rows, batch_autotune
    reqs = [I.compliance_3d(s, n=200003) for s in range(4)]
    say("batch autotune", [p.n for p in reqs])
    probs, xs = [], []
    for p in reqs:
        x = torch.full((p.n,), -1.0, dtype=torch.float32, device="cuda:0")
        probs.append((p.kind, dev(p.y), aligned_rows(dev(p.A)), p.b, p.lo, p.hi, p.C, p.offsets, x))
        xs.append(x)
    torch.cuda.synchronize()
    (s, w), times = batch_autotune(ctx, probs, count=16)
    cand = TUNE_SLOTS
    assert len(times) == len(cand) and all(np.isfinite(t) and t > 0 for t in times), times
    assert s in cand and times[cand.index(s)] == min(times)
    B = Batch(ctx, max_slots=s, wg_per_slot=w, slots_only=True)
    assert B.shape() == (s, w)
    B.close()
    # every request the tuner ran wrote the same bits as a single launch
    for p, x in zip(reqs, xs):
        xs_, _, _ = single(ctx, p)
        assert np.array_equal(x.cpu().numpy(), xs_)


@pytest.mark.parametrize("slots", [2, 8])
def test_server_matches_single_launch_bitwise(ctx, slots):
    from paper_2511_13905_amd.api import Batch
    reqs = [I.compliance_3d(3, n=65537), I.multi_material(2, fields=4, n_per=30001),
            I.volume_com(0, grid=(96, 48)), I.volume_com(1, grid=(64, 32))]
    say("server vs single launch", slots, [p.n for p in reqs])
    st_in = stage(reqs)
    B = Batch(ctx, max_slots=slots)
    handles = [submit(B, p, s) for p, s in zip(reqs, st_in)]
    outs = [collect(B, t, fm, p.n) for (t, fm), p in zip(handles, reqs)]
    B.close()
    for p, (st, r, x, mask, _) in zip(reqs, outs):
        assert st == 0, (p.kind, st)
        xs, rs, ms = single(ctx, p)
        assert np.array_equal(x, xs), p.kind
        assert np.array_equal(mask, ms), p.kind
        assert r["lam"] == rs["lam"] and r["passes"] == rs["passes"], (r, rs)


def test_server_equality_and_automatic_penalty_bitwise(ctx):
    """Equality rows and the automatic penalty through a server slot give the
    bits of a single launch."""
    import dataclasses
    from paper_2511_13905_amd.api import Batch, aligned_rows
    p1 = I.compliance_3d(5, n=40001)
    ax = float(p1.A[0].astype(np.float64) @ np.clip(p1.y.astype(np.float64), p1.lo, p1.hi))
    p1.b = np.array([ax + 0.2 * abs(ax)])                    # equality row lifted to b
    p2 = I.multi_material(4, fields=3, n_per=20011)
    p3 = dataclasses.replace(I.volume_com(2, grid=(64, 32)), C=-1e-7)   # automatic penalty
    cases = [(p1, [True]), (p2, [False, True, False]), (p3, None)]
    say("server equality / automatic penalty", [p.n for p, _ in cases])
    B = Batch(ctx, max_slots=4, slots_only=True)
    staged = []
    for p, eq in cases:
        A = dev(p.A)
        if p.kind != "independent":
            A = aligned_rows(A)
        staged.append((dev(p.y), A))
    torch.cuda.synchronize()
    tickets = [B.submit(p.kind, y, A, p.b, p.lo, p.hi, p.C, offsets=p.offsets, eq=eq)
               for (p, eq), (y, A) in zip(cases, staged)]
    outs = []
    for t in tickets:
        x = B.x_of(t)
        st, r, _ = B.wait(t)
        torch.cuda.synchronize()
        outs.append((st, r, x.cpu().numpy()))
    B.close()
    for (p, eq), (st, r, x) in zip(cases, outs):
        assert st == 0
        xs, rs = ctx.project(p.kind, dev(p.y), dev(p.A), p.b, p.lo, p.hi, p.C, offsets=p.offsets, eq=eq)
        torch.cuda.synchronize()
        assert np.array_equal(x, xs.cpu().numpy()), p.kind
        assert r["lam"] == rs["lam"] and r["kappa"] == rs["kappa"], (r["lam"], rs["lam"])



def test_server_warm_start_bitwise(ctx):
    """Warm-started requests (pgdto_problem.lambda0) through server slots give
    the bits of a warm-started single launch, and the oracle's projection."""
    from paper_2511_13905_amd.api import Batch, aligned_rows
    cases = [I.compliance_3d(6, n=70001), I.multi_material(5, fields=3, n_per=20011),
             I.volume_com(0, grid=(64, 32))]
    refs = [oracle.project(p.kind, p.y, p.A, p.b, p.lo, p.hi, p.C, p.offsets) for p in cases]
    lam0s = [[max(0.0, 0.98 * float(v)) for v in ref.lam] for ref in refs]
    say("server warm start", [p.n for p in cases], lam0s)
    B = Batch(ctx, max_slots=4, slots_only=True)
    staged = []
    for p in cases:
        A = dev(p.A)
        if p.kind != "independent":
            A = aligned_rows(A)
        staged.append((dev(p.y), A))
    torch.cuda.synchronize()
    tickets = [B.submit(p.kind, y, A, p.b, p.lo, p.hi, p.C, offsets=p.offsets, lam0=l0)
               for p, (y, A), l0 in zip(cases, staged, lam0s)]
    outs = []
    for t in tickets:
        x = B.x_of(t)
        st, r, _ = B.wait(t)
        torch.cuda.synchronize()
        outs.append((st, r, x.cpu().numpy()))
    B.close()
    for p, ref, l0, (st, r, x) in zip(cases, refs, lam0s, outs):
        assert st == 0
        xs, rs = ctx.project(p.kind, dev(p.y), dev(p.A), p.b, p.lo, p.hi, p.C, offsets=p.offsets, lam0=l0)
        torch.cuda.synchronize()
        assert np.array_equal(x, xs.cpu().numpy()), p.kind
        assert r["lam"] == rs["lam"] and r["passes"] == rs["passes"], (r["lam"], rs["lam"])
        check(p, x, r, ref)


def test_server_small_slots_stream_block_starts(ctx):
    """Independent blocks on slots of 2 workgroups: most tiles are streamed
    (not held in registers), including the tiles that open a block at an
    unaligned element; masks and x are the bits of a single launch."""
    from paper_2511_13905_amd.api import Batch
    reqs = [I.multi_material(6, fields=3, n_per=40011), I.multi_material(8, fields=4, n_per=25013)]
    say("server small slots", [p.n for p in reqs])
    st_in = stage(reqs)
    B = Batch(ctx, max_slots=8, wg_per_slot=2, slots_only=True)
    handles = [submit(B, p, s) for p, s in zip(reqs, st_in)]
    outs = [collect(B, t, fm, p.n) for (t, fm), p in zip(handles, reqs)]
    B.close()
    for p, (st, r, x, mask, _) in zip(reqs, outs):
        assert st == 0
        xs, rs, ms = single(ctx, p)
        assert np.array_equal(x, xs)
        assert np.array_equal(mask, ms)
        assert r["lam"] == rs["lam"]


def test_server_alone_and_in_mix(ctx):
    """The same request gives the same bits alone and inside a busy mix."""
    from paper_2511_13905_amd.api import Batch
    probe = I.volume_com(4, grid=(128, 64))
    say("alone vs mix", probe.n)
    mix = mixed_requests(7, 30)
    st_probe = stage([probe, probe])
    st_mix = stage(mix)
    # alone in a slot (slots_only), then in the mix of a default executor
    B = Batch(ctx, max_slots=8, slots_only=True)
    t, fm = submit(B, probe, st_probe[0])
    st, r_alone, x_alone, m_alone, _ = collect(B, t, fm, probe.n)
    B.close()
    assert st == 0
    B = Batch(ctx, max_slots=8)
    handles = [submit(B, p, s) for p, s in zip(mix[:15], st_mix[:15])]
    tp, fp = submit(B, probe, st_probe[1])
    handles += [submit(B, p, s) for p, s in zip(mix[15:], st_mix[15:])]
    st, r_mix, x_mix, m_mix, _ = collect(B, tp, fp, probe.n)
    outs = [collect(B, t, fm, p.n) for (t, fm), p in zip(handles, mix)]
    stats = B.stats()
    B.close()
    assert st == 0
    assert np.array_equal(x_alone, x_mix)
    assert np.array_equal(m_alone, m_mix)
    assert r_alone["lam"] == r_mix["lam"]
    ref = oracle.project(probe.kind, probe.y, probe.A, probe.b, probe.lo, probe.hi, probe.C, probe.offsets)
    check(probe, x_mix, r_mix, ref, free_gpu=m_mix)
    assert all(o[0] == 0 for o in outs)
    assert stats["completed"] == 31


def test_server_mix_parity(ctx):
    """A mixed stream of 36 requests, every result against the oracle."""
    from paper_2511_13905_amd.api import Batch
    reqs = mixed_requests(11, 36)
    say("mix parity", len(reqs), sum(p.n for p in reqs))
    st_in = stage(reqs)
    B = Batch(ctx, max_slots=8)
    handles = [submit(B, p, s) for p, s in zip(reqs, st_in)]
    outs = [collect(B, t, fm, p.n) for (t, fm), p in zip(handles, reqs)]
    B.close()
    for p, (st, r, x, mask, times) in zip(reqs, outs):
        assert st == 0, (p.kind, p.n, st)
        assert times[0] <= times[1] <= times[2]
        ref = oracle.project(p.kind, p.y, p.A, p.b, p.lo, p.hi, p.C, p.offsets)
        check(p, x, r, ref, free_gpu=mask)


def test_plain_path_matches(ctx):
    from paper_2511_13905_amd.api import Batch
    reqs = mixed_requests(5, 6)
    say("plain path", [p.n for p in reqs])
    st_in = stage(reqs)
    B = Batch(ctx, max_slots=1)
    handles = [submit(B, p, s) for p, s in zip(reqs, st_in)]
    outs = [collect(B, t, fm, p.n) for (t, fm), p in zip(handles, reqs)]
    B.close()
    for p, (st, r, x, mask, _) in zip(reqs, outs):
        assert st == 0
        xs, rs, ms = single(ctx, p)
        assert np.array_equal(x, xs)
        assert np.array_equal(mask, ms)


def test_server_idle_exit_and_relaunch(ctx):
    """The launch ends after ~50 ms without work; a later request starts it again."""
    from paper_2511_13905_amd.api import Batch
    say("idle relaunch")
    p1 = I.compliance_3d(1, n=20000)
    p2 = I.multi_material(3, fields=4, n_per=5000)
    st_in = stage([p1, p2])
    B = Batch(ctx, max_slots=4, slots_only=True)
    t, fm = submit(B, p1, st_in[0])
    assert collect(B, t, fm, p1.n)[0] == 0
    time.sleep(0.3)
    t, fm = submit(B, p2, st_in[1])
    st, r, x, mask, _ = collect(B, t, fm, p2.n)
    B.close()
    assert st == 0
    ref = oracle.project(p2.kind, p2.y, p2.A, p2.b, p2.lo, p2.hi, p2.C, p2.offsets)
    check(p2, x, r, ref, free_gpu=mask)


def test_server_budget_backpressure(ctx):
    """A tight HBM budget limits the footprint in flight; all requests finish."""
    from paper_2511_13905_amd.api import Batch
    reqs = [I.compliance_3d(s, n=200000) for s in range(6)]
    fp = 4 * 200000 * 3
    say("budget", fp)
    st_in = stage(reqs, mask=False)
    B = Batch(ctx, max_slots=8, hbm_budget_bytes=2 * fp)
    handles = [submit(B, p, s) for p, s in zip(reqs, st_in)]
    outs = [collect(B, t, fm, p.n) for (t, fm), p in zip(handles, reqs)]
    stats = B.stats()
    B.close()
    assert all(o[0] == 0 for o in outs)
    assert stats["peak_bytes"] <= 2 * fp


def test_lone_request_full_gpu_route(ctx):
    """A lone request (nothing else on the device) runs as one full-GPU launch
    by default; the bits equal the slot route and a single launch."""
    from paper_2511_13905_amd.api import Batch
    p = I.multi_material(4, fields=4, n_per=40000)
    say("lone route", p.n)
    st_in = stage([p, p])
    B = Batch(ctx, max_slots=8)
    t, fm = submit(B, p, st_in[0])
    a = collect(B, t, fm, p.n)
    B.close()
    B = Batch(ctx, max_slots=8, slots_only=True)
    t, fm = submit(B, p, st_in[1])
    b = collect(B, t, fm, p.n)
    B.close()
    xs, rs, ms = single(ctx, p)
    assert a[0] == 0 and b[0] == 0
    assert np.array_equal(a[2], b[2]) and np.array_equal(a[2], xs)
    assert np.array_equal(a[3], b[3]) and np.array_equal(a[3], ms)


@pytest.mark.parametrize("slots_only", [False, True])
def test_server_rejects_f64(ctx, slots_only):
    from paper_2511_13905_amd.api import Batch
    from paper_2511_13905_amd import _native as N
    p = I.volume_2d(0)
    say("server f64 request")
    st_in = stage([p])
    B = Batch(ctx, max_slots=2, slots_only=slots_only)
    t, fm = submit(B, p, st_in[0])
    st, r, _ = B.wait(t)
    B.close()
    assert st == N.ERR_ARG


def pgd_states():
    """Two single-row steps (t = 60 and t = 0) and one coupled step."""
    out = [I.pgd_compliance_3d(2, t=60, n=70000), I.pgd_compliance_3d(3, t=0, n=33000)]
    p = I.volume_com(1, grid=(96, 48), vf=0.3)
    rng = np.random.default_rng(5)
    n = p.n
    rho = np.clip(rng.uniform(0, 1, n), I.LO, I.HI).astype(np.float32)
    grad = rng.standard_normal(n).astype(np.float32)
    rho_prev = (rho - 0.01 * rng.standard_normal(n)).astype(np.float32)
    grad_prev = (grad + 0.1 * rng.standard_normal(n)).astype(np.float32)
    A = p.A.astype(np.float32)
    g = A.astype(np.float64) @ rho.astype(np.float64)
    prob = I.Problem("coupled", rho.copy(), A, p.b.copy(), C=p.C)
    out.append(I.PgdState(rho, rho_prev, grad, grad_prev, (-grad_prev).astype(np.float32), prob, g, p.b.copy(), 60))
    return out


def stage_pgd(st):
    from paper_2511_13905_amd.api import aligned_rows
    A = dev(st.problem.A)
    if A.dim() == 1:
        A = A.reshape(1, -1)
    return dict(A=aligned_rows(A), rho=dev(st.rho), rp=dev(st.rho_prev), gr=dev(st.grad), gp=dev(st.grad_prev),
                d=dev(st.d_prev))


@pytest.mark.parametrize("slots_only,warm", [(False, False), (True, False), (True, True)])
def test_served_pgd_steps_match_single_launch(ctx, slots_only, warm):
    """Algorithm 3 steps served (slots or the lone full-GPU route) give the
    bits of pgdto_pgd_step: rho_{t+1}, d_t, alpha, beta, multipliers.  warm:
    both start their projections from the same lambda0 (1.01 x the cold
    step's multipliers), which the served request copies at submit."""
    from paper_2511_13905_amd.api import Batch
    states = pgd_states()
    say("served pgd steps", slots_only, "warm" if warm else "cold", [s.problem.n for s in states])
    lam0s = [None] * len(states)
    if warm:
        for i, st in enumerate(states):
            dv0 = stage_pgd(st)
            _, o0 = ctx.pgd_step(st.problem.kind, dv0["A"], dv0["rho"], dv0["rp"] if st.t > 0 else None, dv0["gr"],
                                 dv0["gp"] if st.t > 0 else None, dv0["d"], st.g, st.G, st.t, I.LO, I.HI,
                                 C=st.problem.C)
            lam0s[i] = [1.01 * max(0.0, v) for v in o0["proj"]["lam"]]
    served = [stage_pgd(s) for s in states]
    single_in = [stage_pgd(s) for s in states]
    torch.cuda.synchronize()
    B = Batch(ctx, max_slots=4, slots_only=slots_only)
    tickets = []
    for st, dv, l0 in zip(states, served, lam0s):
        t = B.submit_pgd(st.problem.kind, dv["A"], dv["rho"], dv["rp"] if st.t > 0 else None, dv["gr"],
                         dv["gp"] if st.t > 0 else None, dv["d"], st.g, st.G, st.t, I.LO, I.HI, C=st.problem.C,
                         lam0=l0)
        tickets.append(t)
    xs = [B.x_of(t) for t in tickets]
    outs = [B.poll_pgd(t, wait=True) for t in tickets]
    B.close()
    torch.cuda.synchronize()
    for st, dv, dv1, x, (status, o, times), l0 in zip(states, served, single_in, xs, outs, lam0s):
        assert status == 0, status
        x1, o1 = ctx.pgd_step(st.problem.kind, dv1["A"], dv1["rho"], dv1["rp"] if st.t > 0 else None, dv1["gr"],
                              dv1["gp"] if st.t > 0 else None, dv1["d"], st.g, st.G, st.t, I.LO, I.HI,
                              C=st.problem.C, lam0=l0)
        torch.cuda.synchronize()
        assert torch.equal(x, x1)
        assert torch.equal(dv["d"], dv1["d"])
        assert o["alpha"] == o1["alpha"] and o["beta"] == o1["beta"]
        assert o["used_fallback"] == o1["used_fallback"] and o["rel_change"] == o1["rel_change"]
        assert o["proj"]["lam"] == o1["proj"]["lam"] and o["proj"]["passes"] == o1["proj"]["passes"]
