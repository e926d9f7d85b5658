"""The autotuners' launch shapes: every 2D transform-pass shape gives bitwise the same
integration, and ridc_autotune records its choice in the tuning table (saved as JSON).

Shape bits: 1 = 64-column waves (FP32/FP64), 2 = 32-wide k-slices (split BF16), 4 = row-major
intermediates folded while staging instead of the prefolded planes (sides that are multiples
of 256)."""
import json
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_1209_4297_amd import ridc
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch, ridc


def _run(env, prob, u0, prec, flags):
    torch, ridc = env
    s = ridc.Ridc(prob, prec=prec)
    s.set_tile(0, 0, flags)
    out = s.integrate(torch.tensor(u0.reshape(-1), device="cuda"), prob["nt"]).cpu().numpy()
    s.close()
    return out


@pytest.mark.parametrize("prec,shapes", [("fp64", [0, 1, 4, 5]), ("fp32", [0, 1, 4, 5]),
                                         ("bf16x3", [0, 2, 4, 6])])
@pytest.mark.parametrize("n", [256, 512, 768])
def test_pass_shapes_are_bitwise_equal(env, prec, shapes, n):
    prob, u0 = workloads.config_reacdiff_2d(n=n, nt=12, order=4, T=0.024)
    print(f"case: 2D n={n} {prec} shapes {shapes}", flush=True)
    ref = _run(env, prob, u0, prec, shapes[0])
    for f in shapes[1:]:
        assert np.array_equal(_run(env, prob, u0, prec, f), ref), f


def test_unavailable_shape_is_rejected(env):
    torch, ridc = env
    prob, _ = workloads.config_reacdiff_2d(n=192, nt=10, order=2, T=0.02)
    s = ridc.Ridc(prob, prec="fp64")
    with pytest.raises(ridc.RidcError):
        s.set_tile(0, 0, 1)        # n = 192: 64-column waves would split the fold
    with pytest.raises(ridc.RidcError):
        s.set_tile(0, 0, 2)        # 32-wide slices are a split-BF16 shape
    with pytest.raises(ridc.RidcError):
        s.set_tile(0, 0, 4)        # n = 192: no prefolded planes, so no choice of them
    s.close()


def test_autotune_records_the_2d_shape(env, tmp_path):
    torch, ridc = env
    prob, u0 = workloads.config_reacdiff_2d(n=256, nt=12, order=4, T=0.024)
    ridc.tune_clear()
    s = ridc.Ridc(prob, prec="bf16x3")
    threads, rows, flags = s.autotune()
    assert flags in (0, 2, 4, 6) and rows == 0 and threads == 512
    x0 = torch.tensor(u0.reshape(-1), device="cuda")
    out = s.integrate(x0, prob["nt"]).cpu().numpy()        # re-armed by integrate
    s.close()
    assert np.array_equal(out, _run(env, prob, u0, "bf16x3", 0))
    path = tmp_path / "tune.json"
    ridc.tune_save(str(path))
    doc = json.loads(path.read_text())
    assert {"n": 256, "prec": 2, "tile": flags} in doc["pass2d"]
    # a second handle of the same key takes the recorded shape without measuring
    s2 = ridc.Ridc(prob, prec="bf16x3")
    assert s2.autotune()[2] == flags
    s2.close()
    ridc.tune_clear()
