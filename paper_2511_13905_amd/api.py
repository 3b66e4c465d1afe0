"""Python binding of the projection library (same names as the C ABI).

Torch tensors provide device memory and streams; the binding only marshals
pointers and sizes into the structs of include/pgdto.h.  Every step of the
projection runs in the HIP kernels of libpgdto.so.
"""
from __future__ import annotations

import atexit
import ctypes as C
import math
import weakref

import torch

from . import _native as N

# Open handles, closed in a fixed order when the interpreter exits (batches,
# whose executor threads and launches use a context's device, before
# contexts), before Python tears down modules and the HIP runtime its own
# exit handlers: no library call is left to a finalizer at shutdown.
_LIVE_BATCHES = weakref.WeakSet()
_LIVE_CONTEXTS = weakref.WeakSet()


def close_all():
    """Close every open Batch, then every open Context, then wait for the device."""
    for b in list(_LIVE_BATCHES):
        b.close()
    for c in list(_LIVE_CONTEXTS):
        c.close()
    if torch.cuda.is_initialized():
        torch.cuda.synchronize()


atexit.register(close_all)


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return N.F32
    if t.dtype == torch.float64:
        return N.F64
    raise TypeError(f"unsupported dtype {t.dtype} (float32 or float64)")


def _check(st: int, where: str):
    if st != N.OK:
        raise N.PgdtoError(st, where)


def make_params(**kw) -> N.Params:
    """pgdto_params with the library defaults, overridden by keyword."""
    p = N.Params()
    N.lib().pgdto_params_default(C.byref(p))
    for k, v in kw.items():
        if k == "search" and isinstance(v, str):
            v = {"newton": N.SEARCH_NEWTON, "bisect": N.SEARCH_BISECT}[v]
        if k == "ncp" and isinstance(v, str):
            v = {"continuous": N.NCP_CONTINUOUS, "paper": N.NCP_PAPER}[v]
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def aligned_rows(A: torch.Tensor) -> torch.Tensor:
    """Return A ([m, n]) with rows on 16-byte boundaries (pads the row stride)."""
    A = A if A.dim() == 2 else A.reshape(1, -1)
    m, n = A.shape
    esz = A.element_size()
    vec = 16 // esz
    if A.stride(1) == 1 and A.data_ptr() % 16 == 0 and (m == 1 or ((A.stride(0) * esz) % 16 == 0 and A.stride(0) >= n)):
        return A                         # one row: its stride is never used
    lda = (n + vec - 1) // vec * vec
    buf = torch.zeros((m, lda), dtype=A.dtype, device=A.device)
    buf[:, :n].copy_(A)
    return buf[:, :n]


class _Keep:
    """Holds host arrays referenced by a struct until the call returns."""

    def __init__(self):
        self.refs = []

    def dbl(self, vals):
        arr = (C.c_double * max(1, len(vals)))(*[float(v) for v in vals])
        self.refs.append(arr)
        return arr

    def i64(self, vals):
        arr = (C.c_int64 * len(vals))(*[int(v) for v in vals])
        self.refs.append(arr)
        return arr


def eq_mask_of(eq) -> int:
    """Equality rows as a bit mask: None, an int mask, or one flag per row/block."""
    if eq is None:
        return 0
    if isinstance(eq, int):
        return eq
    return sum(1 << j for j, e in enumerate(eq) if e)


def problem_struct(kind, y, A, b, lo, hi, C_pen=math.inf, offsets=None, x=None, free_mask=None,
                   keep: _Keep | None = None, copy_ok: bool = True, eq=None, lam0=None):
    """Fill a pgdto_problem from torch tensors; returns (struct, x, A_used).
    copy_ok=False: raise instead of copying A into 16-byte aligned rows.
    eq: rows / blocks held at equality (flags or a bit mask).
    lam0: optional warm-start multipliers, one per row / block."""
    keep = keep or _Keep()
    k = N.KINDS[kind] if isinstance(kind, str) else int(kind)
    if y is not None and not y.is_contiguous():
        raise ValueError("y must be contiguous")
    ref = y if y is not None else x
    n = ref.numel()
    if k == N.INDEPENDENT:
        A_used = A.reshape(-1)
        if not A_used.is_contiguous():
            raise ValueError("independent coefficients must be contiguous")
        m = len(offsets) - 1
        lda = n
    else:
        A_used = aligned_rows(A)
        if not copy_ok and A_used.data_ptr() != A.data_ptr():
            raise ValueError("A rows must start on 16-byte boundaries (stage them with aligned_rows() "
                             "and finish that copy before submitting)")
        m = A_used.shape[0]
        lda = A_used.stride(0) if m > 1 else n
    if x is None:
        x = torch.empty(n, dtype=ref.dtype, device=ref.device)
    s = N.Problem()
    s.kind = k
    s.dtype = _dtype_code(ref)
    s.n = n
    s.m = m
    s.y = y.data_ptr() if y is not None else None
    s.A = A_used.data_ptr()
    s.lda = lda
    s.block_offsets = keep.i64(offsets) if offsets is not None else None
    s.b = keep.dbl(list(b)) if b is not None else None
    s.lo = float(lo)
    s.hi = float(hi)
    s.C = float(C_pen)
    s.x = x.data_ptr()
    s.free_mask = free_mask.data_ptr() if free_mask is not None else None
    s.eq_mask = eq_mask_of(eq)
    s.lambda0 = keep.dbl(list(lam0)) if lam0 is not None else None
    return s, x, A_used


def _stream(device, stream):
    if stream is None:
        return torch.cuda.current_stream(device).cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


class Context:
    """pgdto_ctx: fixed workspace on one device (create once, reuse)."""

    def __init__(self, device: int = 0):
        self.device = device
        h = C.c_void_p()
        _check(N.lib().pgdto_ctx_create(device, C.byref(h)), "pgdto_ctx_create")
        self.h = h
        _LIVE_CONTEXTS.add(self)

    def autotune(self, enable=1) -> int:
        """pgdto_ctx_autotune: grid autotuning per shape class (returns the previous setting)."""
        return N.lib().pgdto_ctx_autotune(self.h, int(enable))

    def autotune_save(self, path: str) -> int:
        """pgdto_ctx_autotune_save: write the tuned grid choices to `path`."""
        n = N.lib().pgdto_ctx_autotune_save(self.h, str(path).encode())
        _check(min(n, 0), "pgdto_ctx_autotune_save")
        return n

    def autotune_load(self, path: str) -> int:
        """pgdto_ctx_autotune_load: add the choices saved in `path` (0 if they
        were measured on another device or library version)."""
        n = N.lib().pgdto_ctx_autotune_load(self.h, str(path).encode())
        _check(min(n, 0), "pgdto_ctx_autotune_load")
        return n

    def trace_passes(self, max_records=128):
        """pgdto_trace_read: the per-pass records of the last one-instance
        launch (a context created with PGDTO_TRACE=1; empty otherwise), as
        dicts of the phase and the device-clock stamps in microseconds from
        the pass start: loop (element loop done), go (the next pass may
        start).  Reading clears the records."""
        import ctypes
        buf = (ctypes.c_uint64 * (8 * max_records))()
        n = N.lib().pgdto_trace_read(self.h, buf, max_records)
        _check(n if n < 0 else 0, "pgdto_trace_read")
        names = {1: "pgd_r", 2: "zero", 3: "search", 4: "stage1", 5: "check", 6: "newton", 7: "final"}
        out = []
        for i in range(n):
            r = list(buf[8 * i:8 * i + 8])
            if r[0] == 0:
                break
            t0 = r[0] & ((1 << 56) - 1)
            end = max(r[4], r[5])
            out.append({"phase": names.get(r[0] >> 56, str(r[0] >> 56)), "loop_us": (r[1] - t0) / 100.0,
                        "pass_us": (end - t0) / 100.0 if end else None})
        return out

    def last_launch(self):
        """(workgroups, tiles) of the last launch on this context."""
        g, t = C.c_int32(), C.c_int32()
        _check(N.lib().pgdto_ctx_last_launch(self.h, C.byref(g), C.byref(t)), "pgdto_ctx_last_launch")
        return g.value, t.value

    def close(self):
        if getattr(self, "h", None):
            N.lib().pgdto_ctx_destroy(self.h)
            self.h = None
            _LIVE_CONTEXTS.discard(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ projection
    def project(self, kind, y, A, b, lo, hi, C=math.inf, offsets=None, x=None, free_mask=None,
                params: N.Params | dict | None = None, stream=None, eq=None, lam0=None):
        """pgdto_project: returns (x, result dict).  Blocks until done.
        eq: rows / blocks held at equality; lam0: warm-start multipliers."""
        keep = _Keep()
        s, x, _A = problem_struct(kind, y, A, b, lo, hi, C, offsets, x, free_mask, keep, eq=eq, lam0=lam0)
        p = params if isinstance(params, N.Params) else make_params(**(params or {}))
        r = N.Result()
        st = N.lib().pgdto_project(self.h, C_byref(s), C_byref(p), C_byref(r), _stream(self.device, stream))
        _check(st, "pgdto_project")
        return x, r.to_dict()

    def project_async(self, kind, y, A, b, lo, hi, result_buf: torch.Tensor, C=math.inf, offsets=None,
                      x=None, free_mask=None, params=None, stream=None, eq=None, lam0=None):
        """pgdto_project_async: enqueue only; the result struct lands in result_buf
        (uint8 device tensor of at least sizeof(pgdto_result) bytes)."""
        keep = _Keep()
        s, x, _A = problem_struct(kind, y, A, b, lo, hi, C, offsets, x, free_mask, keep, eq=eq, lam0=lam0)
        p = params if isinstance(params, N.Params) else make_params(**(params or {}))
        st = N.lib().pgdto_project_async(self.h, C_byref(s), C_byref(p), result_buf.data_ptr(),
                                         _stream(self.device, stream))
        _check(st, "pgdto_project_async")
        return x

    def kappa_path(self, kind, y, A, b, lo, hi, C_values, tau=0.0, offsets=None, x=None, params=None, eq=None,
                   lam0=None, stream=None):
        """pgdto_kappa_path: the projection along a sequence of penalties C,
        each solve warm-started from the previous multipliers; returns (x of
        the last point, [point dicts])."""
        keep = _Keep()
        s, x, _A = problem_struct(kind, y, A, b, lo, hi, math.inf, offsets, x, None, keep, eq=eq, lam0=lam0)
        p = params if isinstance(params, N.Params) else make_params(**(params or {}))
        cs = keep.dbl(list(C_values))
        pts = (N.PathPoint * len(C_values))()
        st = N.lib().pgdto_kappa_path(self.h, C_byref(s), C_byref(p), cs, len(C_values), float(tau), pts,
                                      _stream(self.device, stream))
        _check(st, "pgdto_kappa_path")
        return x, [pt.to_dict(s.m) for pt in pts]

    # ------------------------------------------------------------ Alg. 3 step
    def _pgd_struct(self, kind, A, rho, rho_prev, grad, grad_prev, d, g, G, t, lo, hi, C, offsets, x,
                    hyper, keep, copy_ok=True, eq=None, lam0=None, work=None):
        s, x, _A = problem_struct(kind, None, A, None, lo, hi, C, offsets, x if x is not None else
                                  torch.empty_like(rho), None, keep, copy_ok=copy_ok, eq=eq, lam0=lam0)
        a = N.PgdArgs()
        N.lib().pgdto_pgd_args_default(C_byref(a))
        a.proj = s
        a.rho = rho.data_ptr()
        a.rho_prev = rho_prev.data_ptr() if rho_prev is not None else None
        a.grad = grad.data_ptr()
        a.grad_prev = grad_prev.data_ptr() if grad_prev is not None else None
        a.dir = d.data_ptr()
        a.g = keep.dbl(list(g))
        a.G = keep.dbl(list(G))
        a.t = int(t)
        a.work = work.data_ptr() if work is not None else None
        for k, v in (hyper or {}).items():
            if k == "cg_rule" and isinstance(v, str):
                v = N.CG_RULES[v]
            setattr(a, k, v)
        return a, x

    def pgd_step(self, kind, A, rho, rho_prev, grad, grad_prev, d, g, G, t, lo, hi, C=math.inf,
                 offsets=None, x=None, params=None, stream=None, eq=None, lam0=None, work=None, **hyper):
        """pgdto_pgd_step: one Alg. 3 body.  d is updated in place (d_{t-1} -> d_t);
        returns (rho_{t+1}, out dict).  lam0: warm start of the projection
        (e.g. out["proj"]["lam"] of the previous step); work: optional
        compaction scratch of n elements (may be grad_prev's buffer)."""
        keep = _Keep()
        a, x = self._pgd_struct(kind, A, rho, rho_prev, grad, grad_prev, d, g, G, t, lo, hi, C, offsets, x,
                                hyper, keep, eq=eq, lam0=lam0, work=work)
        p = params if isinstance(params, N.Params) else make_params(**(params or {}))
        out = N.PgdOut()
        st = N.lib().pgdto_pgd_step(self.h, C_byref(a), C_byref(p), C_byref(out), _stream(self.device, stream))
        _check(st, "pgdto_pgd_step")
        return x, out.to_dict()

    # ------------------------------------------------------------ one-launch batches
    def project_batch_async(self, problems, results_buf: torch.Tensor, params=None, slots: int = 0, stream=None):
        """pgdto_project_batch_async: problems is a list of (kind, y, A, b, lo, hi,
        C, offsets, x) tuples (float32, A rows 16-byte aligned, distinct x);
        the result structs land in results_buf (uint8 device tensor of at
        least len(problems) * result_nbytes() bytes)."""
        if results_buf.numel() * results_buf.element_size() < len(problems) * result_nbytes():
            raise ValueError("results_buf holds fewer result structs than problems")
        keep = _Keep()
        arr = (N.Problem * len(problems))()
        for i, (kind, y, A, b, lo, hi, C_pen, offsets, x) in enumerate(problems):
            arr[i], _, _ = problem_struct(kind, y, A, b, lo, hi, C_pen, offsets, x, None, keep, copy_ok=False)
        p = params if isinstance(params, N.Params) else make_params(**(params or {}))
        st = N.lib().pgdto_project_batch_async(self.h, arr, len(problems), C_byref(p), results_buf.data_ptr(),
                                               int(slots), _stream(self.device, stream))
        _check(st, "pgdto_project_batch_async")

    def pgd_step_batch_async(self, steps, outs_buf: torch.Tensor, params=None, slots: int = 0, stream=None):
        """pgdto_pgd_step_batch_async: steps is a list of dicts with the
        arguments of pgd_step (kind, A, rho, rho_prev, grad, grad_prev, d, g, G,
        t, lo, hi, and optionally C, offsets, x and hyper-parameters); x must be
        given.  The pgdto_pgd_out structs land in outs_buf."""
        if outs_buf.numel() * outs_buf.element_size() < len(steps) * result_nbytes(pgd=True):
            raise ValueError("outs_buf holds fewer output structs than steps")
        keep = _Keep()
        arr = (N.PgdArgs * len(steps))()
        for i, s in enumerate(steps):
            s = dict(s)
            hyper = {k: s.pop(k) for k in list(s) if k in ("cg_rule", "t_warmup", "alpha_max", "alpha_fallback",
                                                          "omega", "eps_alpha", "tol_viol", "tol")}
            arr[i], _ = self._pgd_struct(s["kind"], s["A"], s["rho"], s.get("rho_prev"), s["grad"],
                                         s.get("grad_prev"), s["d"], s["g"], s["G"], s["t"], s["lo"], s["hi"],
                                         s.get("C", math.inf), s.get("offsets"), s["x"], hyper, keep,
                                         copy_ok=False, work=s.get("work"))
        p = params if isinstance(params, N.Params) else make_params(**(params or {}))
        st = N.lib().pgdto_pgd_step_batch_async(self.h, arr, len(steps), C_byref(p), outs_buf.data_ptr(), int(slots),
                                                _stream(self.device, stream))
        _check(st, "pgdto_pgd_step_batch_async")

    def pgd_step_async(self, kind, A, rho, rho_prev, grad, grad_prev, d, g, G, t, lo, hi, out_buf,
                       C=math.inf, offsets=None, x=None, params=None, stream=None, lam0=None, work=None, **hyper):
        keep = _Keep()
        a, x = self._pgd_struct(kind, A, rho, rho_prev, grad, grad_prev, d, g, G, t, lo, hi, C, offsets, x,
                                hyper, keep, lam0=lam0, work=work)
        p = params if isinstance(params, N.Params) else make_params(**(params or {}))
        st = N.lib().pgdto_pgd_step_async(self.h, C_byref(a), C_byref(p), out_buf.data_ptr(),
                                          _stream(self.device, stream))
        _check(st, "pgdto_pgd_step_async")
        return x


def project_noalloc(kind, y, A, b, lo, hi, result_buf: torch.Tensor, C=math.inf, offsets=None, x=None,
                    free_mask=None, params=None, stream=None, eq=None, lam0=None):
    """pgdto_project_noalloc: pgdto_project_async with no context (the library's
    static device scratch array is the workspace; the call allocates nothing
    on the device: x must be given, A rows already 16-byte aligned).  Runs on the current device; calls
    that overlap in time on one GPU race.  The result struct lands in
    result_buf (uint8 device tensor of at least sizeof(pgdto_result) bytes)."""
    if x is None:
        raise ValueError("project_noalloc: pass the output x (the call allocates nothing)")
    keep = _Keep()
    s, x, _A = problem_struct(kind, y, A, b, lo, hi, C, offsets, x, free_mask, keep, copy_ok=False, eq=eq,
                              lam0=lam0)
    p = params if isinstance(params, N.Params) else make_params(**(params or {}))
    dev = y.device.index if y.device.index is not None else torch.cuda.current_device()
    st = N.lib().pgdto_project_noalloc(C_byref(s), C_byref(p), result_buf.data_ptr(), _stream(dev, stream))
    _check(st, "pgdto_project_noalloc")
    return x


def C_byref(obj):
    return C.byref(obj)


def result_from_bytes(buf: torch.Tensor, pgd: bool = False) -> dict:
    """Decode a result struct copied back from device memory (uint8 tensor)."""
    raw = bytes(buf.cpu().numpy().tobytes())
    S = N.PgdOut if pgd else N.Result
    obj = S.from_buffer_copy(raw[:C.sizeof(S)])
    return obj.to_dict()


def result_nbytes(pgd: bool = False) -> int:
    return C.sizeof(N.PgdOut if pgd else N.Result)


class Batch:
    """pgdto_batch: continuous batching of projection requests on one device.

    max_slots=1 is the plain one-at-a-time path; otherwise the persistent
    multi-slot executor (float32 streams).  submit() keeps the request's
    tensors alive until the ticket retires; their data must be complete when
    submit() is called (the executor starts at once, in no stream order), so
    it never copies A: rows must already be 16-byte aligned (aligned_rows)."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int = 0, max_slots: int = 0, wg_per_slot: int = 0,
                 queue_capacity: int = 0, slots_only: bool = False):
        cfg = N.BatchCfg()
        cfg.hbm_budget_bytes = int(hbm_budget_bytes)
        cfg.max_slots = int(max_slots)
        cfg.wg_per_slot = int(wg_per_slot)
        cfg.queue_capacity = int(queue_capacity)
        cfg.slots_only = 1 if slots_only else 0
        h = C.c_void_p()
        _check(N.lib().pgdto_batch_create(ctx.h, C.byref(cfg), C.byref(h)), "pgdto_batch_create")
        self.h = h
        self.ctx = ctx
        self._live = {}
        _LIVE_BATCHES.add(self)

    def shape(self):
        s, w = C.c_int32(), C.c_int32()
        _check(N.lib().pgdto_batch_shape(self.h, C.byref(s), C.byref(w)), "pgdto_batch_shape")
        return s.value, w.value

    def submit(self, kind, y, A, b, lo, hi, C=math.inf, offsets=None, x=None, free_mask=None, params=None,
               eq=None, lam0=None) -> int:
        keep = _Keep()
        s, x, A_used = problem_struct(kind, y, A, b, lo, hi, C, offsets, x, free_mask, keep, copy_ok=False, eq=eq,
                                      lam0=lam0)
        p = params if isinstance(params, N.Params) else make_params(**(params or {}))
        t = C_u64()
        _check(N.lib().pgdto_batch_submit(self.h, C_byref(s), C_byref(p), C_byref(t)), "pgdto_batch_submit")
        self._live[t.value] = (y, A_used, x, free_mask)
        return t.value

    def submit_pgd(self, kind, A, rho, rho_prev, grad, grad_prev, d, g, G, t, lo, hi, C=math.inf, offsets=None,
                   x=None, params=None, lam0=None, work=None, **hyper) -> int:
        """pgdto_batch_submit_pgd: one Algorithm 3 step as a served request
        (d is updated in place, rho_{t+1} lands in x).  A must already have
        16-byte aligned rows; the data must be complete when this is called."""
        keep = _Keep()
        a, x = self.ctx._pgd_struct(kind, A, rho, rho_prev, grad, grad_prev, d, g, G, t, lo, hi, C, offsets, x,
                                    hyper, keep, copy_ok=False, lam0=lam0, work=work)
        p = params if isinstance(params, N.Params) else make_params(**(params or {}))
        tk = C_u64()
        _check(N.lib().pgdto_batch_submit_pgd(self.h, C_byref(a), C_byref(p), C_byref(tk)), "pgdto_batch_submit_pgd")
        self._live[tk.value] = (rho, A, x, rho_prev, grad, grad_prev, d, work)
        return tk.value

    def poll_pgd(self, ticket, wait=False):
        """(status, Algorithm 3 output dict or None, times or None)."""
        out = N.PgdOut()
        times = (C.c_int64 * 3)()
        st = N.lib().pgdto_batch_poll_pgd(self.h, ticket, C_byref(out), times, 1 if wait else 0)
        if st in (N.QUEUED, N.PENDING):
            return st, None, None
        self._live.pop(ticket, None)
        return st, out.to_dict(), (times[0], times[1], times[2])

    def x_of(self, ticket):
        return self._live[ticket][2]

    def poll(self, ticket, wait=False):
        """(status, result dict or None, (t_submit, t_start, t_done) ns or None)."""
        r = N.Result()
        times = (C.c_int64 * 3)()
        st = N.lib().pgdto_batch_poll_timed(self.h, ticket, C_byref(r), times, 1 if wait else 0)
        if st in (N.QUEUED, N.PENDING):
            return st, None, None
        self._live.pop(ticket, None)
        return st, r.to_dict(), (times[0], times[1], times[2])

    def wait(self, ticket):
        return self.poll(ticket, wait=True)

    def stats(self):
        v = [C.c_int64() for _ in range(5)]
        _check(N.lib().pgdto_batch_stats(self.h, *[C.byref(x) for x in v]), "pgdto_batch_stats")
        return dict(zip(["admitted", "completed", "queued", "in_flight", "peak_bytes"], [x.value for x in v]))

    def close(self):
        if getattr(self, "h", None):
            N.lib().pgdto_batch_destroy(self.h)
            self.h = None
            self._live.clear()
            _LIVE_BATCHES.discard(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


TUNE_SHAPES = 5                                   # PGDTO_TUNE_SHAPES
TUNE_SLOTS = [4 << c for c in range(TUNE_SHAPES)]   # slot counts of the candidates


def _shape_key(ctx, problems, count):
    """Cache key of an executor-shape choice: library version, device, and the
    kinds, sizes and rows of the samples."""
    props = torch.cuda.get_device_properties(ctx.device)
    dev = f"{getattr(props, 'gcnArchName', props.name)}-{props.multi_processor_count}cu"
    sig = ";".join(f"{k}:{y.numel() if y is not None else x.numel()}:{A.shape[0] if A.dim() > 1 else 1}"
                   for (k, y, A, b, lo, hi, C_pen, offsets, x) in problems)
    return f"v{N.lib().pgdto_version()}|{dev}|{count}|{sig}"


def batch_autotune(ctx: Context, problems, count: int = 64, params=None, cache: str | None = None):
    """pgdto_batch_autotune: the executor shape (slots, workgroups per slot)
    with the highest throughput on `count` requests drawn round-robin from
    `problems` (a list of (kind, y, A, b, lo, hi, C, offsets, x) tuples whose
    tensors are ready), plus the wall time in ms of every candidate shape.
    cache: a JSON file of earlier choices, keyed by library version, device
    and the samples' kinds and sizes; a hit returns the stored shape and
    times without running the candidates, a miss tunes and stores."""
    import json
    import os
    key = _shape_key(ctx, problems, count) if cache else None
    store = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            store = json.load(f)
        if key in store:
            hit = store[key]
            return (int(hit["slots"]), int(hit["wg_per_slot"])), [float(t) for t in hit["times_ms"]]
    shape, times = _batch_autotune_run(ctx, problems, count, params)
    if cache:
        store[key] = {"slots": shape[0], "wg_per_slot": shape[1], "times_ms": times}
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(store, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return shape, times


def _batch_autotune_run(ctx: Context, problems, count: int, params):
    keep = _Keep()
    arr = (N.Problem * len(problems))()
    for i, (kind, y, A, b, lo, hi, C_pen, offsets, x) in enumerate(problems):
        st, _, _ = problem_struct(kind, y, A, b, lo, hi, C_pen, offsets, x, None, keep, copy_ok=False)
        arr[i] = st
    s, w = C.c_int32(), C.c_int32()
    times = (C.c_float * TUNE_SHAPES)()
    pp = params if params is not None else make_params()
    _check(N.lib().pgdto_batch_autotune(ctx.h, arr, len(problems), C.byref(pp), int(count), C.byref(s),
                                        C.byref(w), times), "pgdto_batch_autotune")
    del keep
    return (s.value, w.value), [float(t) for t in times]


def C_u64():
    return C.c_uint64()
