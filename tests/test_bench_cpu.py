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
    for key, (src, sha, nbytes) in bench.MEASURED_TRAFFIC.items():
        assert src in bench.KERNEL_SOURCE
        assert len(sha) == 16 and nbytes > 0
        current = bench.code_hash(bench.KERNEL_SOURCE[src])
        expect = nbytes if current == sha else None
        assert bench.measured_traffic(*key) == expect


def test_code_hash_ignores_comments_and_blank_space_only(bench, tmp_path):
    a, b, c = tmp_path / "a.hip", tmp_path / "b.hip", tmp_path / "c.hip"
    a.write_text("int f(int x) {\n  return x + 1;  // one\n}\n")
    b.write_text("/* doc */ int f(int x)\n{ return x + 1; }\n// trailing\n")
    c.write_text("int f(int x) {\n  return x + 2;\n}\n")
    assert bench.code_hash(str(a)) == bench.code_hash(str(b))
    assert bench.code_hash(str(a)) != bench.code_hash(str(c))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr)


@pytest.mark.parametrize("prec,products", [("fp64", 1), ("fp32", 1), ("bf16x3", 3)])
def test_pass_roofline_counts_the_folded_issued_work(bench, prec, products):
    """A folded pass (n a multiple of 64) issues n^3 flops per level (three BF16 products per
    folded one in the split-BF16 pass): the frac is that work over the dtype's peak, so a pass
    running exactly at peak reads 1.0, and the plain 2 n^3 count is a labelled extra."""
    n, levels = 1024, 4
    dense = 2.0 * n**3 * levels
    issued = n**3 * levels * products
    peak = bench.MFMA_PEAK_TFLOPS[prec]
    us_at_peak = issued / (peak * 1e12) * 1e6
    r = bench.roofline_pass(us_at_peak, dense, n, prec)
    assert r["flops_per_launch"] == issued and r["dense_flops_per_launch"] == dense
    assert abs(r["frac"] - 1.0) < 1e-4
    r = bench.roofline_pass(2 * us_at_peak, dense, n, prec)
    assert abs(r["frac"] - 0.5) < 1e-4 and r["peak"] == peak
    # an unfolded side (n % 64 != 0) issues the plain product
    r = bench.roofline_pass(1.0, 2.0 * 96**3, 96, prec)
    assert r["flops_per_launch"] == 2.0 * 96**3 * products
