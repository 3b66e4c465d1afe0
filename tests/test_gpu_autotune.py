"""Grid autotuner: the chosen workgroup count changes the speed, never the bits."""
import numpy as np
import pytest

from paper_2511_13905_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


@pytest.mark.parametrize("gen", ["single", "independent", "coupled"])
def test_autotune_bitwise(gen):
    from paper_2511_13905_amd.api import Context
    p = {"single": lambda: I.compliance_3d(4, n=600000),
         "independent": lambda: I.multi_material(1, fields=4, n_per=150000),
         "coupled": lambda: I.volume_com(2, grid=(128, 64, 32))}[gen]()
    print("[case] autotune", gen, p.n, flush=True)
    y, A = dev(p.y), dev(p.A)
    plain = Context(0)
    x0, r0 = plain.project(p.kind, y, A, p.b, p.lo, p.hi, p.C, offsets=p.offsets)
    g0, tiles = plain.last_launch()
    plain.close()
    tuned = Context(0)
    assert tuned.autotune(1) == 0
    x1, r1 = tuned.project(p.kind, y, A, p.b, p.lo, p.hi, p.C, offsets=p.offsets)   # tunes, then runs
    g1, tiles1 = tuned.last_launch()
    x2, r2 = tuned.project(p.kind, y, A, p.b, p.lo, p.hi, p.C, offsets=p.offsets)   # uses the choice
    g2, _ = tuned.last_launch()
    assert tuned.autotune(-1) == 1
    tuned.close()
    torch.cuda.synchronize()
    assert tiles1 == tiles
    assert g1 == g2 and g2 in {max(1, g0 // k) for k in (1, 2, 4, 8)}
    assert torch.equal(x0, x1) and torch.equal(x0, x2)
    assert r0["lam"] == r1["lam"] == r2["lam"]


def test_autotune_choices_persist(tmp_path):
    """Grid choices saved by one context are loaded by another (same device,
    same library version) and used without tuning again; a file written for
    another device is ignored."""
    from paper_2511_13905_amd.api import Context
    p = I.compliance_3d(5, n=700000)
    print("[case] autotune persist", p.n, flush=True)
    y, A = dev(p.y), dev(p.A)
    a = Context(0)
    a.autotune(1)
    a.project(p.kind, y, A, p.b, p.lo, p.hi)
    g_tuned, _ = a.last_launch()
    path = str(tmp_path / "grid.tune")
    assert a.autotune_save(path) >= 1
    a.close()
    b = Context(0)                      # autotuning off: only the loaded choice can set the grid
    assert b.autotune_load(path) >= 1
    b.project(p.kind, y, A, p.b, p.lo, p.hi)
    assert b.last_launch()[0] == g_tuned
    text = open(path).read().splitlines()
    other = str(tmp_path / "other.tune")
    with open(other, "w") as f:
        f.write(text[0].rsplit(" ", 1)[0] + " gfx000-1cu\n" + "\n".join(text[1:]) + "\n")
    c = Context(0)
    assert c.autotune_load(other) == 0
    b.close()
    c.close()


def test_executor_shape_cache(tmp_path):
    """batch_autotune with a cache file: the first call tunes and stores, the
    second returns the stored shape without running the candidates."""
    import time
    from paper_2511_13905_amd.api import Context, aligned_rows, batch_autotune
    ctx = Context(0)
    probs = []
    for s in range(4):
        p = I.compliance_3d(s, n=200000)
        x = torch.empty(p.n, dtype=torch.float32, device="cuda:0")
        probs.append((p.kind, dev(p.y), aligned_rows(dev(p.A)), p.b, p.lo, p.hi, p.C, None, x))
    print("[case] executor shape cache", len(probs), flush=True)
    torch.cuda.synchronize()
    cache = str(tmp_path / "shapes.json")
    shape1, t1 = batch_autotune(ctx, probs, count=16, cache=cache)
    t0 = time.perf_counter()
    shape2, t2 = batch_autotune(ctx, probs, count=16, cache=cache)
    hit_s = time.perf_counter() - t0
    ctx.close()
    assert shape2 == shape1 and t2 == t1
    assert hit_s < 0.05
