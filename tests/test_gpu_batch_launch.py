"""GPU tests of the one-launch batch entry points (pgdto_project_batch_async,
pgdto_pgd_step_batch_async): every instance of a batch must give the bits of
its own one-instance launch (same solver, tile-ordered reductions), whatever
the slot count; a sample is also held to the oracle.  Every case prints its
name and shapes before touching the GPU."""
import numpy as np
import pytest

import oracle
from paper_2511_13905_amd import _native as N
from paper_2511_13905_amd import inputs as I

from parity import check

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


def mixed_problems():
    return [I.compliance_3d(0, n=300_001), I.compliance_3d(1, n=4_096), I.multi_material(2, n_per=65_536),
            I.volume_com(0, grid=(48, 24, 24)), I.volume_com(1, grid=(48, 24, 24)), I.compliance_3d(3, n=77_777),
            I.multi_material(4, fields=3, n_per=10_007), I.volume_com(2, grid=(64, 32)),
            I.compliance_3d(5, n=1_000_000), I.volume_com(3, grid=(40, 20))]


def field_diff(a: bytes, b: bytes, pgd=False):
    """Names (and values) of the struct fields whose bytes differ."""
    import ctypes as C
    S = N.PgdOut if pgd else N.Result
    out = []

    def walk(S, off, prefix):
        for name, typ in S._fields_:
            fo = getattr(S, name).offset + off
            if isinstance(typ, type) and issubclass(typ, C.Structure):
                walk(typ, fo, prefix + name + ".")
                continue
            sz = C.sizeof(typ)
            if a[fo:fo + sz] != b[fo:fo + sz]:
                va, vb = typ.from_buffer_copy(a[fo:fo + sz]), typ.from_buffer_copy(b[fo:fo + sz])
                if hasattr(va, "__len__"):
                    es = C.sizeof(typ._type_)
                    idx = [k for k in range(len(va)) if a[fo + k * es:fo + (k + 1) * es] != b[fo + k * es:fo + (k + 1) * es]]
                    out.append((prefix + name, [(k, va[k], vb[k]) for k in idx[:8]]))
                else:
                    out.append((prefix + name, va.value, vb.value))
    walk(S, 0, "")
    return out


def staged(p):
    from paper_2511_13905_amd.api import aligned_rows
    y = dev(p.y)
    A = dev(p.A)
    if p.kind != "independent":
        A = aligned_rows(A)
    return y, A


@pytest.mark.parametrize("slots", [0, 3, 10])
def test_project_batch_matches_single_launches(ctx, slots):
    from paper_2511_13905_amd.api import result_nbytes, result_from_bytes
    probs = mixed_problems()
    say("project-batch", f"slots={slots}", [(p.kind, p.n, p.m) for p in probs])
    staged_all = [staged(p) for p in probs]
    xs_b = [torch.full_like(y, float("nan")) for y, _ in staged_all]
    xs_s = [torch.empty_like(y) for y, _ in staged_all]
    nb = result_nbytes()
    res_b = torch.zeros(nb * len(probs), dtype=torch.uint8, device="cuda:0")
    res_s = torch.zeros(nb * len(probs), dtype=torch.uint8, device="cuda:0")
    torch.cuda.synchronize()
    ctx.project_batch_async([(p.kind, y, A, p.b, p.lo, p.hi, p.C, p.offsets, x)
                             for p, (y, A), x in zip(probs, staged_all, xs_b)], res_b, slots=slots)
    torch.cuda.synchronize()
    for i, (p, (y, A), x) in enumerate(zip(probs, staged_all, xs_s)):
        ctx.project_async(p.kind, y, A, p.b, p.lo, p.hi, res_s[i * nb:(i + 1) * nb], C=p.C, offsets=p.offsets, x=x)
    torch.cuda.synchronize()
    for i, p in enumerate(probs):
        rb = result_from_bytes(res_b[i * nb:(i + 1) * nb])
        assert rb["error"] == 0, (i, rb)
        assert torch.equal(xs_b[i], xs_s[i]), f"instance {i} ({p.kind}, n={p.n}): x differs"
        ra = bytes(res_b[i * nb:(i + 1) * nb].cpu().numpy().tobytes())
        rs = bytes(res_s[i * nb:(i + 1) * nb].cpu().numpy().tobytes())
        assert ra == rs, f"instance {i} ({p.kind}, n={p.n}): result differs (batch, single): {field_diff(ra, rs)}"
    # the oracle on two of them (a single row and a coupled infeasible seed)
    for i in (1, 4):
        p = probs[i]
        ref = oracle.project(p.kind, p.y, p.A, p.b, p.lo, p.hi, p.C, p.offsets)
        check(p, xs_b[i].cpu().numpy(), result_from_bytes(res_b[i * nb:(i + 1) * nb]), ref)


def test_pgd_step_batch_matches_single_steps(ctx):
    from paper_2511_13905_amd.api import result_nbytes, result_from_bytes
    states = [I.pgd_compliance_3d(s, t=(0 if s == 2 else 60), n=n) for s, n in
              ((0, 200_003), (1, 65_536), (2, 30_000), (3, 500_000), (4, 4_096), (5, 123_457))]
    say("pgd-batch", [(st.rho.size, st.t) for st in states])
    steps_b, steps_s = [], []
    for st in states:
        base = dict(kind="single", A=dev(st.problem.A), rho=dev(st.rho), rho_prev=dev(st.rho_prev), grad=dev(st.grad),
                    grad_prev=dev(st.grad_prev), g=st.g, G=st.G, t=st.t, lo=I.LO, hi=I.HI)
        steps_b.append(dict(base, d=dev(st.d_prev), x=torch.full_like(base["rho"], float("nan"))))
        steps_s.append(dict(base, d=dev(st.d_prev), x=torch.empty_like(base["rho"])))
    nb = result_nbytes(pgd=True)
    out_b = torch.zeros(nb * len(states), dtype=torch.uint8, device="cuda:0")
    out_s = torch.zeros(nb * len(states), dtype=torch.uint8, device="cuda:0")
    torch.cuda.synchronize()
    ctx.pgd_step_batch_async(steps_b, out_b, slots=4)
    torch.cuda.synchronize()
    for i, s in enumerate(steps_s):
        ctx.pgd_step_async(s["kind"], s["A"], s["rho"], s["rho_prev"], s["grad"], s["grad_prev"], s["d"], s["g"],
                           s["G"], s["t"], s["lo"], s["hi"], out_s[i * nb:(i + 1) * nb], x=s["x"])
    torch.cuda.synchronize()
    for i in range(len(states)):
        ob = result_from_bytes(out_b[i * nb:(i + 1) * nb], pgd=True)
        assert ob["proj"]["error"] == 0, (i, ob)
        assert torch.equal(steps_b[i]["x"], steps_s[i]["x"]), f"step {i}: rho_next differs"
        assert torch.equal(steps_b[i]["d"], steps_s[i]["d"]), f"step {i}: direction differs"
        ra = bytes(out_b[i * nb:(i + 1) * nb].cpu().numpy().tobytes())
        rs = bytes(out_s[i * nb:(i + 1) * nb].cpu().numpy().tobytes())
        assert ra == rs, f"step {i}: output differs (batch, single): {field_diff(ra, rs, pgd=True)}"
    st = states[4]
    ref = oracle.pgd_step("single", st.rho, st.rho_prev, st.grad, st.grad_prev, st.d_prev, st.problem.A, st.g, st.G,
                          st.t, I.LO, I.HI, stream_dtype=np.float32)
    ob = result_from_bytes(out_b[4 * nb:5 * nb], pgd=True)
    assert abs(ob["alpha"] - ref["alpha"]) <= 1e-12 * abs(ref["alpha"])
    xg = steps_b[4]["x"].cpu().numpy().astype(np.float64)
    assert np.max(np.abs(xg - ref["proj"].x) / np.abs(ref["proj"].x)) <= 1e-5


def test_batch_rejects_bad_lists(ctx):
    import ctypes as C
    from paper_2511_13905_amd.api import make_params, problem_struct, _Keep
    say("batch-bad-lists")
    p64 = I.volume_2d(0)
    y, A = staged(p64)
    keep = _Keep()
    arr = (N.Problem * 1)()
    arr[0], _, _ = problem_struct(p64.kind, y, A, p64.b, p64.lo, p64.hi, p64.C, None, torch.empty_like(y), None, keep)
    prm = make_params()
    res = torch.zeros(4096, dtype=torch.uint8, device="cuda:0")
    stream = torch.cuda.current_stream().cuda_stream
    L = N.lib()
    assert L.pgdto_project_batch_async(ctx.h, arr, 1, C.byref(prm), res.data_ptr(), 0, stream) == N.ERR_ARG   # float64
    assert L.pgdto_project_batch_async(ctx.h, arr, 0, C.byref(prm), res.data_ptr(), 0, stream) == N.ERR_ARG
    assert L.pgdto_project_batch_async(ctx.h, arr, N.BATCH_MAX + 1, C.byref(prm), res.data_ptr(), 0,
                                       stream) == N.ERR_ARG
    torch.cuda.synchronize()


def test_batch_and_single_launches_repeat_bitwise(ctx):
    """The same list twice through the batch launch (3 slots), and each
    instance twice through one-instance launches: bitwise repeats."""
    from paper_2511_13905_amd.api import result_nbytes
    probs = mixed_problems()
    say("repeat", [(p.kind, p.n) for p in probs])
    st = [staged(p) for p in probs]
    nb = result_nbytes()
    outs = []
    for rep in range(2):
        xs = [torch.empty_like(y) for y, _ in st]
        res = torch.zeros(nb * len(probs), dtype=torch.uint8, device="cuda:0")
        ctx.project_batch_async([(p.kind, y, A, p.b, p.lo, p.hi, p.C, p.offsets, x)
                                 for p, (y, A), x in zip(probs, st, xs)], res, slots=3)
        torch.cuda.synchronize()
        outs.append((xs, bytes(res.cpu().numpy().tobytes())))
    for i in range(len(probs)):
        assert torch.equal(outs[0][0][i], outs[1][0][i]), f"batch repeat: x of instance {i} differs"
        a, b = outs[0][1][i * nb:(i + 1) * nb], outs[1][1][i * nb:(i + 1) * nb]
        assert a == b, f"batch repeat: instance {i} result differs: {field_diff(a, b)}"
    for i, (p, (y, A)) in enumerate(zip(probs, st)):
        rr = []
        for rep in range(2):
            x = torch.empty_like(y)
            res = torch.zeros(nb, dtype=torch.uint8, device="cuda:0")
            ctx.project_async(p.kind, y, A, p.b, p.lo, p.hi, res, C=p.C, offsets=p.offsets, x=x)
            torch.cuda.synchronize()
            rr.append((x, bytes(res.cpu().numpy().tobytes())))
        assert torch.equal(rr[0][0], rr[1][0]), f"single repeat: x of instance {i} differs"
        assert rr[0][1] == rr[1][1], f"single repeat: instance {i} result differs: {field_diff(rr[0][1], rr[1][1])}"
