"""CPU tests of bench.py's host side: the one-GPU refusal, the algorithmic
byte models behind roofline.bytes_per_launch, and the rule that measured
traffic is reported only for the kernel sources it was measured on."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
N_C1 = 256 * 128 * 128


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_pgd_step_bytes_per_pass_kind():
    # pass R (5 streams), zero pass (4 read + 2 written), 5 search passes (2 each), final (3 + 1):
    # 25 float32 streams = 100 bytes per element at 8 passes
    r = {"iters_search": 5, "passes": 8, "n_compact": -1, "passes_compacted": 0}
    assert bench.pgd_bytes(N_C1, r) == N_C1 * 100
    assert bench.pgd_bytes(N_C1, r) * 16 == 6_710_886_400          # the 16-instance launch
    r6 = dict(r, iters_search=6)
    assert bench.pgd_bytes(N_C1, r6) - bench.pgd_bytes(N_C1, r) == N_C1 * 8


def test_projection_bytes():
    # every pass reads y and the rows, the final pass also writes x
    r = {"iters_search": 5, "passes": 7, "n_compact": -1, "passes_compacted": 0}
    assert bench.proj_bytes(N_C1, 1, r) == 7 * N_C1 * 8 + N_C1 * 4
    rc = {"iters_search": 0, "passes": 13, "n_compact": -1, "passes_compacted": 0}   # coupled, m = 5
    assert bench.proj_bytes(1_769_472, 5, rc) == 13 * 1_769_472 * 24 + 1_769_472 * 4


def test_compacted_pairs_count_once_written_and_read_per_later_pass():
    kept, pc = 1000, 3
    r = {"iters_search": 5, "passes": 8, "n_compact": kept, "passes_compacted": pc}
    full = {"iters_search": 5, "passes": 8, "n_compact": -1, "passes_compacted": 0}
    # pc of the search passes stream only the kept pairs (written once, read pc times)
    assert bench.pgd_bytes(N_C1, full) - bench.pgd_bytes(N_C1, r) == pc * N_C1 * 8 - kept * 8 * (1 + pc)


def test_measured_traffic_only_for_the_measured_sources(monkeypatch):
    sha = bench.MEASURED_TRAFFIC["pgd_compliance"]["kernel_sha"]
    monkeypatch.setattr(bench, "kernel_sha", lambda files=None: sha)
    t = bench.traffic_for("pgd_compliance", 16)
    assert t is not None and t["read"] + t["written"] == t["bytes_per_launch"]
    monkeypatch.setattr(bench, "kernel_sha", lambda files=None: "0" * 16)
    assert bench.traffic_for("pgd_compliance", 16) is None
    assert bench.traffic_for("project_compliance", 16) is None


def test_kernel_sha_is_stable():
    a, b = bench.kernel_sha(), bench.kernel_sha()
    assert a == b and len(a) == 16 and int(a, 16) >= 0
    assert bench.kernel_sha(bench.WIDE_SRC) != a
