"""Host-side checks of the C ABI library (no GPU work): it loads, exports every declared entry
point, and its host plan (exact weights, PCR stage plan, footprints) is right."""
import math
import os
import re
from fractions import Fraction

import pytest

from oracle import lagrange_integral_weights

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def ridc():
    from paper_1209_4297_amd import ridc as mod
    return mod


def test_header_symbols_are_exported(ridc):
    text = open(os.path.join(ROOT, "include", "ridc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(ridc_[a-z_0-9]+)\s*\(", text))
    assert len(names) >= 15
    for name in sorted(names):
        assert hasattr(ridc.lib(), name), name
    assert set(ridc.EXPORTED) == names


@pytest.mark.parametrize("j", range(1, 12))
def test_library_weights_are_correctly_rounded(ridc, j):
    for r in range(j):
        exact = lagrange_integral_weights(list(range(j + 1)), r, r + 1)
        got = ridc.quadrature_weights(j, r)
        assert got == [float(x) for x in exact], (j, r)


def test_weights_reject_bad_rows(ridc):
    with pytest.raises(ridc.RidcError):
        ridc.quadrature_weights(3, 3)
    with pytest.raises(ridc.RidcError):
        ridc.quadrature_weights(0, 0)


def _dense_cyclic_solve_check(r, m, stages, divisor):
    """Apply the PCR plan's stage recursion in exact-ish float arithmetic to a cyclic system and
    compare with a dense solve (numpy), for small m."""
    import numpy as np
    a = np.zeros((m, m))
    for i in range(m):
        a[i, i] += 1 + 2 * r
        a[i, (i - 1) % m] += -r
        a[i, (i + 1) % m] += -r
    d = np.random.default_rng(m).standard_normal(m)
    x_ref = np.linalg.solve(a, d)
    # replay the stages: coefficients b, c of the cyclic system with stride s
    b, c = 1 + 2 * r, -r
    s = 1
    for _ in range(stages):
        g = c / b
        d = d - g * (np.roll(d, s) + np.roll(d, -s))
        b, c = b - 2 * c * c / b, -c * c / b
        s = (2 * s) % m
    x = d / divisor
    return np.max(np.abs(x - x_ref)) / np.max(np.abs(x_ref))


@pytest.mark.parametrize("r,m", [(0.2, 128), (33.6, 16386), (1e4, 64), (1e4, 100), (0.0, 10),
                                 (5.0, 2), (3.0, 7), (1e6, 1000)])
def test_pcr_plan(ridc, r, m):
    stages, divisor = ridc.pcr_plan(r, m)
    if r == 0:
        assert stages == 0 and divisor == 1.0
        return
    if m <= 2000:
        # both solves lose accuracy with the condition number 1 + 4r
        assert _dense_cyclic_solve_check(r, m, stages, divisor) < 1e-14 * (10 + 4 * r)
    # a system whose coupling decays fast needs few stages
    if r < 1:
        assert stages <= 8


def test_footprint(ridc):
    import workloads
    prob, _ = workloads.config_reacdiff_1d()
    fp = ridc.footprint_bytes(prob)
    # 17 ring slots of 8192 doubles for order 4 (3 + 5 + 7 + 2), plus small tables
    assert 17 * 8192 * 8 <= fp < 17 * 8192 * 8 + 64 * 1024
    bad = dict(prob, n=1)
    assert ridc.footprint_bytes(bad) == 0


@pytest.mark.parametrize("change,code", [
    (dict(n=1), -1), (dict(dt=0.0), -1), (dict(dt=float("nan")), -1), (dict(order=0), -1),
    (dict(order=13), -1), (dict(nu=-1.0), -1), (dict(length=0.0), -1), (dict(dim=3), -1),
    (dict(bc=7), -1), (dict(fe_kind=9), -1), (dict(prec=5), -1), (dict(reserved=1), -1),
    (dict(dim=2, bc=0), -2), (dict(dim=2, n=100), -2), (dict(dim=2, fe_kind=1), -2),
    (dict(dim=1, prec=1), -2),
])
def test_create_rejects_bad_problems_before_touching_the_device(ridc, change, code):
    import ctypes
    import workloads
    prob, _ = workloads.config_reacdiff_1d()
    p = ridc.make_problem(prob)
    for k, v in change.items():
        setattr(p, k, v)
    h = ctypes.c_void_p()
    rc = ridc.lib().ridc_create(ctypes.byref(p), None, ctypes.byref(h))
    assert rc == code
    assert not h.value
    assert ridc.lib().ridc_last_error()                      # a message for the caller
    assert ridc.lib().ridc_footprint_bytes(ctypes.byref(p)) == 0


def test_null_safety(ridc):
    lib = ridc.lib()
    assert lib.ridc_destroy(None) == 0
    assert lib.ridc_remaining(None) == -1
    assert lib.ridc_sync(None) == ridc.RIDC_E_INVAL
    assert lib.ridc_read(None, None, None) == ridc.RIDC_E_INVAL
    assert lib.ridc_advance(None, 0, 5) == 0


def test_batch_tile_validation(ridc):
    lib = ridc.lib()
    for threads, rows in [(128, 0), (300, 0), (256, -1), (256, 100)]:
        assert lib.ridc_set_batch_tile(threads, rows) == ridc.RIDC_E_INVAL
    for threads, rows in [(1024, 768), (512, 0), (256, 0)]:
        assert lib.ridc_set_batch_tile(threads, rows) == 0
    assert lib.ridc_autotune_batch(None, 1, None, None) == ridc.RIDC_E_INVAL


def test_noalloc_rejects_before_any_device_work(ridc):
    """The allocation-free entry point checks its arguments and the size of its fixed array on
    the host first: these calls return before any pointer is touched (no GPU needed)."""
    import ctypes
    lib = ridc.lib()
    fake = ctypes.c_void_p(0x1000)     # never dereferenced: every case fails on the host
    base = dict(dim=1, bc="periodic", n=128, length=2 * math.pi, fe="advect", order=4, a=1.0,
                nu=0.1, T=1.0, nt=200)
    cases = [
        (dict(base, n=1 << 20), ridc.RIDC_E_UNSUPPORTED),     # 17 slots x 8 MiB > 32 MiB
        (dict(base, order=7), ridc.RIDC_E_UNSUPPORTED),
        (dict(base, dim=2, bc="dirichlet", fe="none", n=64), ridc.RIDC_E_UNSUPPORTED),
        (dict(base, nu=-1.0), ridc.RIDC_E_INVAL),
    ]
    for prob, code in cases:
        p = ridc.make_problem(prob)
        rc = lib.ridc_integrate_noalloc(ctypes.byref(p), None, fake, 10, fake, None)
        assert rc == code, (prob, rc, lib.ridc_last_error())
    p = ridc.make_problem(base)
    assert lib.ridc_integrate_noalloc(ctypes.byref(p), None, fake, 2, fake, None) == \
        ridc.RIDC_E_INVAL                                     # fewer than order-1 steps
    assert lib.ridc_integrate_noalloc(ctypes.byref(p), None, None, 10, fake, None) == \
        ridc.RIDC_E_INVAL


@pytest.mark.parametrize("pair", ["fbe", "ark3", "ark4"])
def test_stage_weights_are_correctly_rounded(ridc, pair):
    """The IMEX corrector's interpolation and partial-interval weights (host plan, exact
    integer arithmetic) are the correctly rounded exact values for every window size, start-up
    position and stage abscissa."""
    from oracle import ridc_ext as X
    tab = X.SCHEMES[pair]
    for S in range(2, 13):
        for r in range(S - 1):
            nodes = list(range(S))
            for i in range(tab.s):
                li, qi = ridc.stage_weights(S, r, pair, i)
                t = Fraction(r) + tab.c[i]
                lx = X._lagrange_values(nodes, t)
                qx = lagrange_integral_weights(nodes, Fraction(r), t)
                assert li == [float(v) for v in lx], (S, r, i)
                assert qi == [float(v) for v in qx], (S, r, i)


def test_ext_validation_and_footprint(ridc):
    """ridc_create_ext's host checks: reactions need Dirichlet grids, n <= 8192, the top order
    <= 12; the footprint counts the value and f rings, weights and stage workspaces."""
    import ctypes
    lib = ridc.lib()
    base = dict(dim=1, bc="dirichlet", n=1000, length=1.0, fe="none", order=2, a=0.0, nu=1e-3,
                T=1.0, nt=100, fi="cubic", kappa=10.0, pairs=["ark3", "fbe"])
    assert ridc.footprint_bytes(base) > 0
    assert ridc.footprint_bytes(dict(base, bc="periodic")) == 0
    assert ridc.footprint_bytes(dict(base, n=8193)) == 0
    assert ridc.footprint_bytes(dict(base, order=3, pairs=["ark4", "ark4", "ark4"])) > 0
    assert ridc.footprint_bytes(dict(base, order=4, pairs=["ark4"] * 4)) == 0    # order 16
    p = ridc.make_problem(base)
    e = ridc.make_ext(base)
    out = ctypes.c_void_p()
    assert lib.ridc_create_ext(ctypes.byref(p), None, None, ctypes.byref(out)) == \
        ridc.RIDC_E_INVAL
    e.reserved = 1
    assert lib.ridc_create_ext(ctypes.byref(p), ctypes.byref(e), None, ctypes.byref(out)) == \
        ridc.RIDC_E_INVAL


def test_tune_cache_round_trip(ridc, tmp_path):
    """The tuning table's file format: entries loaded from a file are written back unchanged
    (1D tilings, the grouped tiling, 2D pass shapes); unreadable files are errors."""
    import json
    doc = {"format": "ridc-tune-1", "device": "",
           "tile1d": [{"n": 8192, "bc": 1, "stages": 13, "threads": 1024, "rows": 128,
                       "flags": 1},
                      {"n": 128, "bc": 0, "stages": 7, "threads": 512, "rows": 0, "flags": 2}],
           "batch1d": {"threads": 512, "rows": 1536},
           "pass2d": [{"n": 1024, "prec": 2, "tile": 2}, {"n": 512, "prec": 0, "tile": 1}]}
    src = tmp_path / "in.json"
    src.write_text(json.dumps(doc))
    ridc.tune_clear()
    ridc.tune_load(str(src))
    out = tmp_path / "sub" / "out.json"
    ridc.tune_save(str(out))
    got = json.loads(out.read_text())
    assert got["format"] == "ridc-tune-1"
    for key in ("tile1d", "pass2d"):
        assert sorted(got[key], key=json.dumps) == sorted(doc[key], key=json.dumps)
    assert got["batch1d"] == doc["batch1d"]
    ridc.tune_clear()
    ridc.tune_save(str(out))
    assert json.loads(out.read_text())["tile1d"] == []
    with pytest.raises(ridc.RidcError):
        ridc.tune_load(str(tmp_path / "missing.json"))
