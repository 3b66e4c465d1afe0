"""GPU tests of the free-set compaction of the 1-D searches (Sec. 4.2.1:
saturated variables contribute nothing to the Jacobian, so once the bracket
is narrow their terms are folded into per-tile sums and only the undecided
elements are streamed).  Compaction on and off must both meet the oracle's
bar; with it on, every route (one-instance launch, batch launch, served
slot) must give the same bits; tiles that cannot be compacted (more than
half of them undecided) must fall back.  Compaction is opt-in
(pgdto_params.compact = 1).  Every case prints its name first."""
import numpy as np
import pytest

import oracle
from paper_2511_13905_amd import inputs as I

from parity import check, free_from_mask

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


CASES = {
    "single-f32": lambda: I.compliance_3d(0, n=1_048_576),
    "single-f32-ragged": lambda: I.compliance_3d(3, n=999_983),
    "single-f64": lambda: I.compliance_3d(1, n=524_288, dtype=np.float64),
    "independent": lambda: I.multi_material(2, n_per=262_144),
    "independent-uneven": lambda: I.multi_material(4, fields=3, n_per=100_003),
}


def run(ctx, p, compact, eq=None):
    from paper_2511_13905_amd.api import aligned_rows
    y = dev(p.y)
    A = dev(p.A) if p.kind == "independent" else aligned_rows(dev(p.A))
    mask = torch.zeros((p.n + 31) // 32, dtype=torch.int32, device="cuda:0")
    x, r = ctx.project(p.kind, y, A, p.b, p.lo, p.hi, p.C, offsets=p.offsets, free_mask=mask,
                       params={"compact": compact}, eq=eq)
    torch.cuda.synchronize()
    return x.cpu().numpy(), r, free_from_mask(mask.cpu().numpy().view(np.uint32), p.n)


@pytest.mark.parametrize("case", list(CASES))
def test_compaction_meets_the_oracle(ctx, case):
    p = CASES[case]()
    say("compaction", case, p.kind, p.n, p.m, p.y.dtype)
    ref = oracle.project(p.kind, p.y, p.A, p.b, p.lo, p.hi, p.C, p.offsets)
    x1, r1, f1 = run(ctx, p, 1)
    x0, r0, f0 = run(ctx, p, 0)
    check(p, x1, r1, ref, f1)
    check(p, x0, r0, ref, f0)
    assert r0["n_compact"] == -1
    # the bracket narrows to a few percent: a small fraction is kept
    assert 0 <= r1["n_compact"] < 0.25 * p.n, r1["n_compact"]
    assert r1["n_compact"] > 0
    rel = np.max(np.abs(x1.astype(np.float64) - x0) / np.abs(ref.x))
    assert rel <= 1e-5, rel


def test_compaction_equality_row(ctx):
    p = I.compliance_3d(6, n=600_000)
    p.b = p.b * 1.05                # the equality target lies above a.clip(y): the row is lowered
    say("compaction equality row", p.n)
    ref = oracle.project(p.kind, p.y, p.A, p.b, p.lo, p.hi, p.C, p.offsets, eq=[True])
    x1, r1, f1 = run(ctx, p, 1, eq=[True])
    check(p, x1, r1, ref, f1)
    assert r1["n_compact"] > 0


def test_compaction_dense_breakpoints(ctx):
    """Breakpoints packed into a relative width of about 1e-8 around the root:
    at the compaction pass about half of every tile is undecided, which
    exercises tiles kept whole (more than half undecided) beside compacted
    ones; the result must still meet the oracle's bar."""
    n = 1 << 20
    rng = np.random.default_rng(7)
    y = (0.5 + 1e-9 * rng.standard_normal(n)).astype(np.float64)
    a = np.full(n, -1.0 / n)
    lam = 0.5 * n                   # z = y + 0.5: about half of the elements above the box
    x = np.clip(y - lam * a, I.LO, I.HI)
    b = np.array([float(np.sum(a * x))])
    p = I.Problem("single", y, a.reshape(1, n), b)
    say("compaction dense breakpoints", n)
    ref = oracle.project(p.kind, p.y, p.A, p.b, p.lo, p.hi, p.C)
    x1, r1, f1 = run(ctx, p, 1)
    check(p, x1, r1, ref, f1)
    assert r1["n_compact"] <= n // 2, r1["n_compact"]


def test_compaction_routes_bitwise(ctx):
    """Compaction on: the one-instance launch, a batch launch and a served
    slot give the same bits (the compaction depends on the tiles' data only)."""
    from paper_2511_13905_amd.api import Batch, aligned_rows, result_nbytes, result_from_bytes
    probs = [I.compliance_3d(8, n=1_048_576), I.multi_material(9, n_per=200_000), I.compliance_3d(10, n=300_000)]
    say("compaction routes", [(p.kind, p.n) for p in probs])
    st = []
    for p in probs:
        A = dev(p.A) if p.kind == "independent" else aligned_rows(dev(p.A))
        st.append((dev(p.y), A))
    on = {"compact": 1}
    single = []
    for p, (y, A) in zip(probs, st):
        x, r = ctx.project(p.kind, y, A, p.b, p.lo, p.hi, p.C, offsets=p.offsets, params=on)
        assert r["n_compact"] > 0
        single.append((x, r))
    nb = result_nbytes()
    res = torch.zeros(nb * len(probs), dtype=torch.uint8, device="cuda:0")
    xb = [torch.empty_like(y) for y, _ in st]
    ctx.project_batch_async([(p.kind, y, A, p.b, p.lo, p.hi, p.C, p.offsets, x)
                             for p, (y, A), x in zip(probs, st, xb)], res, slots=2, params=on)
    torch.cuda.synchronize()
    B = Batch(ctx, max_slots=4, slots_only=True)
    tk = [B.submit(p.kind, y, A, p.b, p.lo, p.hi, p.C, p.offsets, params=on) for p, (y, A) in zip(probs, st)]
    served = []
    for t in tk:
        x = B.x_of(t)
        stt, r, _ = B.wait(t)
        assert stt == 0
        served.append((x, r))
    B.close()
    torch.cuda.synchronize()
    for i, p in enumerate(probs):
        rb = result_from_bytes(res[i * nb:(i + 1) * nb])
        assert torch.equal(xb[i], single[i][0]), f"batch x differs ({p.kind})"
        assert torch.equal(served[i][0], single[i][0]), f"served x differs ({p.kind})"
        for k in ("lam", "resid", "n_compact", "passes", "n_free"):
            assert rb[k] == single[i][1][k] == served[i][1][k], (k, p.kind)


def test_pgd_step_with_work_buffer(ctx):
    """An Algorithm 3 step compacts into its work buffer: same oracle bar as
    without, and the buffer may be the caller's grad_prev."""
    st = I.pgd_compliance_3d(11, t=60, n=1_048_576)
    say("pgd work buffer", st.rho.size)
    ref = oracle.pgd_step("single", st.rho, st.rho_prev, st.grad, st.grad_prev, st.d_prev, st.problem.A, st.g, st.G,
                          st.t, I.LO, I.HI, stream_dtype=np.float32)
    outs = []
    for work in ("none", "own", "grad_prev"):
        A, rho, rp, gr, gp = dev(st.problem.A), dev(st.rho), dev(st.rho_prev), dev(st.grad), dev(st.grad_prev)
        d = dev(st.d_prev)
        wb = {"none": None, "own": torch.empty_like(rho), "grad_prev": gp}[work]
        x, out = ctx.pgd_step("single", A, rho, rp, gr, gp, d, st.g, st.G, st.t, I.LO, I.HI, work=wb,
                              params={"compact": 1})
        torch.cuda.synchronize()
        xv = x.cpu().numpy().astype(np.float64)
        assert np.max(np.abs(xv - ref["proj"].x) / np.abs(ref["proj"].x)) <= 1e-5, work
        assert abs(out["alpha"] - ref["alpha"]) <= 1e-12 * abs(ref["alpha"])
        assert (out["proj"]["n_compact"] > 0) == (work != "none"), (work, out["proj"]["n_compact"])
        outs.append((x, out))
    assert torch.equal(outs[1][0], outs[2][0])


def test_compaction_is_off_by_default(ctx):
    p = I.compliance_3d(12, n=400_000)
    say("compaction default off", p.n)
    y, A = dev(p.y), dev(p.A)
    _, r = ctx.project(p.kind, y, A, p.b, p.lo, p.hi)
    assert r["n_compact"] == -1 and r["passes_compacted"] == 0
