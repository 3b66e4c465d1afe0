"""GPU checks at the largest sizes: more than 2^31 elements per problem.

Element indices, tile bounds, block offsets and free-mask words are 64-bit
in the kernels; these cases put every one of them past 2^31 (a ragged n, a
block boundary and a tile boundary beyond it).  The oracle cannot solve
2^31 elements in seconds, so the checks are the ones that hold at any size:

- the multipliers against planted ones: b_j is a_j . clip(y - A^T lam_p)
  summed in float64, so with kappa = 0 the exact solution is lam_p (eq. (h),
  Theorem 1; unique because the free set is not empty);
- x on sampled elements against the oracle's clip map at the returned
  multipliers (all of the ragged tail, the first elements and those around
  2^31 and the block boundary are in the sample);
- the free-mask bits on the same sample against the oracle's z, away from a
  1e-6 band around the bounds, and zero bits past n;
- a_j . x - b_j over the whole stored x, summed in float64 by torch, against
  the reported residual and against zero;
- the reported free count against the float64 count of free z, up to the
  elements in the band, and against the mask's popcount (exactly).

Inputs: seeded on the device (torch's Philox generator), the compliance
recipe's distributions: y = u - 0.1 g with u ~ U(0,1), g ~ N(0,1);
compliance row a = -(|N(0,1)| + 0.01); the coupled second row is a
uniform volume row of ones.
"""
import numpy as np
import pytest

from oracle import projection as P

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

LO, HI = 1e-3, 1.0
EDGE = 1 << 31
N_BIG = EDGE + 4099                # ragged: not a multiple of 4 or 32
CHUNK = 1 << 27
BAND = 1e-6
DEV = "cuda:0"


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2511_13905_amd.api import Context
    c = Context(0)
    yield c
    c.close()


def say(*a):
    print("[case]", *a, flush=True)


def chunks(s0, s1):
    for s in range(s0, s1, CHUNK):
        yield s, min(s1, s + CHUNK)


def gen_inputs(seed, n, dtype, rows):
    """y and the coefficient rows ([rows, lda] with lda a multiple of 4)."""
    dev = DEV
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    lda = (n + 3) // 4 * 4
    y = torch.empty(n, dtype=dtype, device=dev)
    A = torch.zeros((rows, lda), dtype=dtype, device=dev)
    for s, e in chunks(0, n):
        k = e - s
        u = torch.rand(k, generator=g, device=dev, dtype=torch.float64)
        gg = torch.randn(k, generator=g, device=dev, dtype=torch.float64)
        y[s:e] = (u - 0.1 * gg).to(dtype)
        A[0, s:e] = (-(torch.randn(k, generator=g, device=dev, dtype=torch.float64).abs() + 0.01)).to(dtype)
    if rows > 1:
        A[1, :n] = 1.0
    return y, A[:, :n]


def z_of(y, A, lam, s, e):
    """z = y - A^T lam on [s, e) in float64 (A rows given per element range)."""
    z = y[s:e].double()
    for j, l in enumerate(lam):
        z = z - l * A[j, s:e].double()
    return z


def popcount(words):
    w = words.to(torch.int64) & 0xFFFFFFFF
    c = torch.zeros((), dtype=torch.int64, device=words.device)
    for k in range(32):
        c += ((w >> k) & 1).sum()
    return int(c)


CASES = [
    # (kind, dtype, planted multipliers)
    ("single", torch.float32, [0.3]),
    ("independent", torch.float32, [0.3, 0.1]),
    ("coupled", torch.float32, [0.3, 0.2]),
    ("single", torch.float64, [0.2]),
]


@pytest.mark.parametrize("kind,dtype,lam_p", CASES, ids=lambda v: str(v).replace("torch.", ""))
def test_beyond_2_31_elements(ctx, kind, dtype, lam_p):
    n = N_BIG
    seed = 31
    say("large", kind, str(dtype), "n", n, "seed", seed, "planted", lam_p)
    rows = 2 if kind == "coupled" else 1
    y, A = gen_inputs(seed, n, dtype, rows)
    split = EDGE - 5
    if kind == "independent":
        offsets = [0, split, n]
        # block j: z = y - lam_j a on its own elements
        b = []
        for j in range(2):
            acc = 0.0
            for s, e in chunks(offsets[j], offsets[j + 1]):
                z = y[s:e].double() - lam_p[j] * A[0, s:e].double()
                acc += float((A[0, s:e].double() * z.clamp(LO, HI)).sum())
            b.append(acc)
    else:
        offsets = None
        b = [0.0] * rows
        for s, e in chunks(0, n):
            xp = z_of(y, A, lam_p, s, e).clamp(LO, HI)
            for j in range(rows):
                b[j] += float((A[j, s:e].double() * xp).sum())
    mask = torch.zeros((n + 31) // 32, dtype=torch.int32, device=DEV)
    # rows as [rows, n] views with a 16-byte aligned stride (no staging copy)
    coef = A[0] if kind == "independent" else A
    x, r = ctx.project(kind, y, coef, b, LO, HI, offsets=offsets, free_mask=mask)
    if DEV != "cpu":
        torch.cuda.synchronize()
    print("outcome", r["outcome"], "passes", r["passes"], "lam", r["lam"], "n_free", r["n_free"], flush=True)
    assert r["outcome"] == "converged"
    m = len(lam_p)
    lam = np.array(r["lam"][:m])
    assert np.allclose(lam, lam_p, rtol=1e-6, atol=0), (lam, lam_p)

    # residuals and the free count over the whole array, float64
    resid = [0.0] * m
    nfree = nband = 0
    segs = [(0, offsets[1]), (offsets[1], n)] if kind == "independent" else [(0, n)]
    for jseg, (s0, s1) in enumerate(segs):
        for s, e in chunks(s0, s1):
            if kind == "independent":
                z = y[s:e].double() - lam[jseg] * A[0, s:e].double()
            else:
                z = z_of(y, A, lam, s, e)
            nfree += int(((z >= LO) & (z <= HI)).sum())
            nband += int((((z - LO).abs() <= BAND) | ((z - HI).abs() <= BAND)).sum())
            xs = x[s:e].double()
            if kind == "independent":
                resid[jseg] += float((A[0, s:e].double() * xs).sum())
            else:
                for j in range(m):
                    resid[j] += float((A[j, s:e].double() * xs).sum())
    for j in range(m):
        rj = resid[j] - b[j]
        tol = 1e-6 * abs(b[j])
        assert abs(r["resid"][j] - rj) <= tol, (j, r["resid"][j], rj, tol)
        assert abs(rj) <= tol, (j, rj, tol)
    assert abs(r["n_free"] - nfree) <= nband, (r["n_free"], nfree, nband)
    assert popcount(mask) == r["n_free"]
    last = int(mask[-1].item()) & 0xFFFFFFFF
    assert last >> (n % 32) == 0, hex(last)

    # sampled elements against the oracle's clip map
    rng = np.random.default_rng(seed)
    idx = np.unique(np.concatenate([rng.integers(0, n, 1 << 16), np.arange(64), np.arange(n - 4200, n),
                                    np.arange(EDGE - 64, EDGE + 64), np.arange(split - 64, split + 64)]))
    ti = torch.from_numpy(idx).to(DEV)
    ys = y.index_select(0, ti).double().cpu().numpy()
    As = np.stack([A[j].index_select(0, ti).double().cpu().numpy() for j in range(rows)])
    xs = x.index_select(0, ti).double().cpu().numpy()
    words = mask.index_select(0, torch.from_numpy(idx >> 5).to(DEV)).cpu().numpy().astype(np.uint32)
    bits = ((words >> (idx & 31).astype(np.uint32)) & 1).astype(bool)
    if kind == "independent":
        xr = np.empty_like(ys)
        zr = np.empty_like(ys)
        for j, (s0, s1) in enumerate(segs):
            sel = (idx >= s0) & (idx < s1)
            xr[sel], zr[sel] = P.clip_map(ys[sel], As[:, sel], [lam[j]], LO, HI)
    else:
        xr, zr = P.clip_map(ys, As, lam, LO, HI)
    xerr = float(np.max(np.abs(xs - xr) / np.abs(xr)))
    assert xerr <= 1e-5, xerr
    far = np.minimum(np.abs(zr - LO), np.abs(zr - HI)) > BAND
    free_ref = (zr >= LO) & (zr <= HI)
    assert not np.any((bits != free_ref) & far)
    print("xerr", xerr, "sampled", idx.size, "band", nband, flush=True)
    del x, y, A, mask, coef
    if DEV != "cpu":
        torch.cuda.empty_cache()
