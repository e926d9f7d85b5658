"""Host-side checks of bench.py: the byte accounting behind its roofline and the one-GPU guard."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


@pytest.fixture(scope="module")
def bench():
    import bench as mod
    return mod


@pytest.mark.parametrize("P,vectors", [(1, 2), (2, 9), (3, 17), (4, 26)])
def test_method_step_bytes_counts_stored_windows(bench, P, vectors):
    # level 0: eta read, eta/F/C written; middle level j: eta, j+1 F and one C read, three
    # written; top level: P+2 read, eta written (a single level reads and writes eta)
    assert bench.method_step_bytes(P, 1) == 8 * vectors
    assert bench.method_step_bytes(P, 8192) == 8 * vectors * 8192


def test_method_step_bytes_by_level_sum(bench):
    for P in range(2, 9):
        levels = [4] + [j + 6 for j in range(1, P - 1)] + [P + 3]
        assert bench.method_step_bytes(P, 3) == 8 * 3 * sum(levels)


def test_traffic_table_is_tied_to_source_hashes(bench):
    import hashlib
    for key, (src, sha, nbytes) in bench.MEASURED_TRAFFIC.items():
        assert src in bench.KERNEL_SOURCE
        assert len(sha) == 16 and nbytes > 0
        with open(bench.KERNEL_SOURCE[src], "rb") as f:
            current = hashlib.sha256(f.read()).hexdigest()[:16]
        expect = nbytes if current == sha else None
        assert bench.measured_traffic(*key) == expect


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr)
