"""Thin ctypes binding of the RIDC C ABI (``include/ridc.h``).

Argument marshalling only: every step of the integration runs in the HIP library.  Device
arrays are torch CUDA float64 tensors; work runs on the current torch stream unless a stream
is given.  There is no CPU fallback: importing this module raises if ``libridc.so`` is absent.
"""
from __future__ import annotations

import ctypes
import math
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_PKG, "libridc.so")

RIDC_OK = 0
RIDC_E_INVAL = -1
RIDC_E_UNSUPPORTED = -2
RIDC_E_NOMEM = -3
RIDC_E_HIP = -4
RIDC_E_NONFINITE = -5
RIDC_E_STATE = -6

BC = {"periodic": 0, "dirichlet": 1}
FE = {"none": 0, "advect": 1, "logistic": 2, "upwind": 3, "burgers": 4}
PREC = {"fp64": 0, "fp32": 1, "bf16x3": 2}

_ERR_NAMES = {-1: "RIDC_E_INVAL", -2: "RIDC_E_UNSUPPORTED", -3: "RIDC_E_NOMEM",
              -4: "RIDC_E_HIP", -5: "RIDC_E_NONFINITE", -6: "RIDC_E_STATE"}


class RidcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_ERR_NAMES.get(code, code)}: {msg}")
        self.code = code


class Problem(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32), ("bc", ctypes.c_int32), ("n", ctypes.c_int64),
        ("length", ctypes.c_double), ("fe_kind", ctypes.c_int32), ("order", ctypes.c_int32),
        ("a", ctypes.c_double), ("nu", ctypes.c_double), ("dt", ctypes.c_double),
        ("prec", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


FS = {"diffusion": 0, "logistic": 1, "cubic": 2}
PAIR = {"fbe": 0, "ark3": 1, "ark4": 2}


class Ext(ctypes.Structure):
    _fields_ = [
        ("fs_kind", ctypes.c_int32), ("newton_maxit", ctypes.c_int32), ("kappa", ctypes.c_double),
        ("pair", ctypes.c_int32 * 12), ("reserved", ctypes.c_int32),
    ]


def _load():
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"RIDC HIP library not built: {_LIB_PATH} is missing "
                          "(run paper_1209_4297_amd/build.py)")
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    sig = {
        "ridc_create": (ctypes.c_int, [ctypes.POINTER(Problem), vp, ctypes.POINTER(vp)]),
        "ridc_destroy": (ctypes.c_int, [vp]),
        "ridc_footprint_bytes": (ctypes.c_size_t, [ctypes.POINTER(Problem)]),
        "ridc_integrate": (ctypes.c_int, [vp, dp, i64, dp, dp]),
        "ridc_integrate_batch": (ctypes.c_int, [ctypes.POINTER(vp), i32, ctypes.POINTER(vp),
                                                ctypes.POINTER(i64), ctypes.POINTER(vp)]),
        "ridc_begin": (ctypes.c_int, [vp, dp, i64]),
        "ridc_advance": (ctypes.c_int, [ctypes.POINTER(vp), i32, i64]),
        "ridc_remaining": (i64, [vp]),
        "ridc_read": (ctypes.c_int, [vp, dp, dp]),
        "ridc_sync": (ctypes.c_int, [vp]),
        "ridc_last_error": (ctypes.c_char_p, []),
        "ridc_quadrature_weights": (ctypes.c_int, [i32, i32, ctypes.POINTER(ctypes.c_double)]),
        "ridc_pcr_plan": (ctypes.c_int, [ctypes.c_double, i64, ctypes.POINTER(i32),
                                         ctypes.POINTER(ctypes.c_double)]),
        "ridc_step_cost": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_double)]),
        "ridc_version": (ctypes.c_char_p, []),
        "ridc_autotune": (ctypes.c_int, [vp, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                         ctypes.POINTER(i32)]),
        "ridc_set_tile": (ctypes.c_int, [vp, i32, i32, i32]),
        "ridc_kernel_time": (ctypes.c_int, [vp, i32, ctypes.POINTER(ctypes.c_double),
                                            ctypes.POINTER(ctypes.c_double)]),
        "ridc_integrate_restarts": (ctypes.c_int, [vp, dp, i64, i32, dp]),
        "ridc_set_batch_tile": (ctypes.c_int, [i32, i32]),
        "ridc_stencil_time": (ctypes.c_int, [vp, i32, ctypes.POINTER(ctypes.c_double),
                                             ctypes.POINTER(ctypes.c_double)]),
        "ridc_batch_kernel_time": (ctypes.c_int, [ctypes.POINTER(vp), i32, i32,
                                                  ctypes.POINTER(ctypes.c_double),
                                                  ctypes.POINTER(ctypes.c_double)]),
        "ridc_autotune_batch": (ctypes.c_int, [ctypes.POINTER(vp), i32, ctypes.POINTER(i32),
                                               ctypes.POINTER(i32)]),
        "ridc_integrate_noalloc": (ctypes.c_int, [ctypes.POINTER(Problem), vp, dp, i64, dp,
                                                  vp]),
        "ridc_create_ext": (ctypes.c_int, [ctypes.POINTER(Problem), ctypes.POINTER(Ext), vp,
                                           ctypes.POINTER(vp)]),
        "ridc_footprint_bytes_ext": (ctypes.c_size_t, [ctypes.POINTER(Problem),
                                                       ctypes.POINTER(Ext)]),
        "ridc_stage_weights": (ctypes.c_int, [i32, i32, i32, i32,
                                              ctypes.POINTER(ctypes.c_double),
                                              ctypes.POINTER(ctypes.c_double)]),
        "ridc_tune_save": (ctypes.c_int, [ctypes.c_char_p]),
        "ridc_tune_load": (ctypes.c_int, [ctypes.c_char_p]),
        "ridc_tune_clear": (ctypes.c_int, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()
EXPORTED = ("ridc_create", "ridc_destroy", "ridc_footprint_bytes", "ridc_integrate",
            "ridc_integrate_batch", "ridc_begin", "ridc_advance", "ridc_remaining", "ridc_read",
            "ridc_sync", "ridc_last_error", "ridc_quadrature_weights", "ridc_pcr_plan",
            "ridc_step_cost", "ridc_version", "ridc_autotune", "ridc_set_tile",
            "ridc_kernel_time", "ridc_integrate_restarts", "ridc_set_batch_tile",
            "ridc_autotune_batch", "ridc_batch_kernel_time", "ridc_stencil_time",
            "ridc_integrate_noalloc", "ridc_create_ext", "ridc_footprint_bytes_ext",
            "ridc_stage_weights", "ridc_tune_save", "ridc_tune_load", "ridc_tune_clear")


def lib():
    return _lib


def library_path() -> str:
    return _LIB_PATH


def _check(rc: int):
    if rc != RIDC_OK:
        raise RidcError(rc, _lib.ridc_last_error().decode())


def make_problem(prob: dict, dt: float | None = None, prec: str = "fp64") -> Problem:
    """ctypes ``ridc_problem`` from a workload dictionary (see ``workloads``)."""
    if dt is None:
        dt = float(prob["T"]) / int(prob["nt"])
    return Problem(dim=int(prob["dim"]), bc=BC[prob["bc"]], n=int(prob["n"]),
                   length=float(prob["length"]), fe_kind=FE[prob["fe"]],
                   order=int(prob["order"]), a=float(prob.get("a", 0.0)),
                   nu=float(prob["nu"]), dt=float(dt), prec=PREC[prec], reserved=0)


def uses_ext(prob: dict) -> bool:
    """True for workloads with IMEX levels (``pairs``) or a stiff reaction (``fi``)."""
    return "pairs" in prob or prob.get("fi", "diffusion") != "diffusion"


def make_ext(prob: dict, newton_maxit: int = 0) -> Ext:
    """ctypes ``ridc_ext`` from a workload dictionary: ``pairs`` (one of fbe/ark3/ark4 per
    level; default forward-backward Euler everywhere), ``fi`` (diffusion, logistic or cubic:
    the stiff term nu Lap_h + kappa g) and ``kappa``."""
    order = int(prob["order"])
    pairs = prob.get("pairs", ["fbe"] * order)
    if len(pairs) != order:
        raise ValueError("one pair per level is needed")
    arr = (ctypes.c_int32 * 12)(*[PAIR[x] for x in pairs])
    return Ext(fs_kind=FS[prob.get("fi", "diffusion")], newton_maxit=int(newton_maxit),
               kappa=float(prob.get("kappa", 0.0)), pair=arr, reserved=0)


def footprint_bytes(prob: dict, dt: float | None = None, prec: str = "fp64") -> int:
    p = make_problem(prob, dt, prec)
    if uses_ext(prob):
        e = make_ext(prob)
        return int(_lib.ridc_footprint_bytes_ext(ctypes.byref(p), ctypes.byref(e)))
    return int(_lib.ridc_footprint_bytes(ctypes.byref(p)))


def stage_weights(S: int, r: int, pair: str, stage: int):
    """(interp, quad) weights of an IMEX corrector stage on a window of S nodes."""
    li = (ctypes.c_double * S)()
    qi = (ctypes.c_double * S)()
    _check(_lib.ridc_stage_weights(int(S), int(r), PAIR[pair], int(stage), li, qi))
    return list(li), list(qi)


def quadrature_weights(j: int, r: int):
    out = (ctypes.c_double * (j + 1))()
    _check(_lib.ridc_quadrature_weights(j, r, out))
    return list(out)


def pcr_plan(r: float, m: int):
    st = ctypes.c_int32()
    dv = ctypes.c_double()
    _check(_lib.ridc_pcr_plan(r, m, ctypes.byref(st), ctypes.byref(dv)))
    return st.value, dv.value


def _ptr(t):
    if t is None:
        return None
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
            and t.is_contiguous()):
        raise TypeError("device arrays must be contiguous float64 CUDA tensors")
    return ctypes.c_void_p(t.data_ptr())


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Ridc:
    """One RIDC integrator instance (owns its device rings, transforms and workspaces)."""

    def __init__(self, prob: dict, dt: float | None = None, prec: str = "fp64", stream=None,
                 newton_maxit: int = 0):
        self.prob = dict(prob)
        self.prec = prec
        self._p = make_problem(prob, dt, prec)
        self.order = self._p.order
        self.npts = self._p.n if self._p.dim == 1 else self._p.n * self._p.n
        self.side = self._p.n
        self._h = ctypes.c_void_p()
        self._stream = stream
        if uses_ext(prob):
            self._e = make_ext(prob, newton_maxit)
            _check(_lib.ridc_create_ext(ctypes.byref(self._p), ctypes.byref(self._e),
                                        _stream_ptr(stream), ctypes.byref(self._h)))
        else:
            _check(_lib.ridc_create(ctypes.byref(self._p), _stream_ptr(stream),
                                    ctypes.byref(self._h)))

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            _lib.ridc_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def integrate(self, u0, nsteps: int, uT=None, levels=None, sync: bool = True):
        import torch
        if uT is None:
            uT = torch.empty_like(u0)
        _check(_lib.ridc_integrate(self._h, _ptr(u0), int(nsteps), _ptr(uT), _ptr(levels)))
        if sync:
            self.sync()
        return uT

    def integrate_restarts(self, u0, nsteps: int, segments: int, uT=None, sync: bool = True):
        import torch
        if uT is None:
            uT = torch.empty_like(u0)
        _check(_lib.ridc_integrate_restarts(self._h, _ptr(u0), int(nsteps), int(segments),
                                            _ptr(uT)))
        if sync:
            self.sync()
        return uT

    def begin(self, u0, nsteps: int):
        _check(_lib.ridc_begin(self._h, _ptr(u0), int(nsteps)))

    def remaining(self) -> int:
        return int(_lib.ridc_remaining(self._h))

    def read(self, uT, levels=None):
        _check(_lib.ridc_read(self._h, _ptr(uT), _ptr(levels)))

    def sync(self):
        _check(_lib.ridc_sync(self._h))

    def autotune(self):
        """Pick the fastest tiling (1D); the handle must be re-armed afterwards.
        Returns (threads, rows, flags)."""
        t = ctypes.c_int32()
        r = ctypes.c_int32()
        f = ctypes.c_int32()
        _check(_lib.ridc_autotune(self._h, ctypes.byref(t), ctypes.byref(r), ctypes.byref(f)))
        return t.value, r.value, f.value

    def set_tile(self, threads: int, rows: int, flags: int = 0):
        _check(_lib.ridc_set_tile(self._h, int(threads), int(rows), int(flags)))

    def kernel_time(self, reps: int = 50):
        """(us per launch, algorithmic work per launch) of the dominant kernel at the next
        pipeline step (bytes for 1D, flops for 2D)."""
        us = ctypes.c_double()
        w = ctypes.c_double()
        _check(_lib.ridc_kernel_time(self._h, int(reps), ctypes.byref(us), ctypes.byref(w)))
        return us.value, w.value

    def stencil_time(self, reps: int = 50):
        """2D: (us per launch, algorithmic bytes per launch) of the right-hand-side kernel at
        the next pipeline step."""
        us = ctypes.c_double()
        b = ctypes.c_double()
        _check(_lib.ridc_stencil_time(self._h, int(reps), ctypes.byref(us), ctypes.byref(b)))
        return us.value, b.value

    def step_cost(self):
        b = ctypes.c_double()
        f = ctypes.c_double()
        _check(_lib.ridc_step_cost(self._h, ctypes.byref(b), ctypes.byref(f)))
        return b.value, f.value


def _handle_array(solvers):
    arr = (ctypes.c_void_p * len(solvers))()
    for i, s in enumerate(solvers):
        arr[i] = s.handle.value
    return arr


def advance(solvers, max_steps: int):
    """Advance several instances together (grouped launches per pipeline step)."""
    _check(_lib.ridc_advance(_handle_array(solvers), len(solvers), int(max_steps)))


def integrate_batch(solvers, u0s, nsteps, uTs):
    n = len(solvers)
    u0a = (ctypes.c_void_p * n)(*[t.data_ptr() for t in u0s])
    uTa = (ctypes.c_void_p * n)(*[t.data_ptr() for t in uTs])
    nsa = (ctypes.c_int64 * n)(*[int(x) for x in nsteps])
    _check(_lib.ridc_integrate_batch(_handle_array(solvers), n, u0a, nsa, uTa))


def set_batch_tile(threads: int, rows: int):
    """Tiling of grouped 1D launches: threads per workgroup and the most LDS rows per workgroup
    (0: whole cycles).  Process-wide; results do not depend on it."""
    _check(_lib.ridc_set_batch_tile(int(threads), int(rows)))


def autotune_batch(solvers):
    """Measure the grouped-launch tilings on these instances and keep the fastest; returns
    (threads, rows).  The instances are left unarmed."""
    t, r = ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.ridc_autotune_batch(_handle_array(solvers), len(solvers), ctypes.byref(t),
                                    ctypes.byref(r)))
    return t.value, r.value


def batch_kernel_time(solvers, reps: int):
    """(us per grouped launch, algorithmic bytes per launch) of the armed instances' next step."""
    us, b = ctypes.c_double(), ctypes.c_double()
    _check(_lib.ridc_batch_kernel_time(_handle_array(solvers), len(solvers), int(reps),
                                       ctypes.byref(us), ctypes.byref(b)))
    return us.value, b.value


def integrate_noalloc(prob: dict, u0, nsteps: int, uT=None, nonfinite=None, dt=None,
                      stream=None):
    """1D integration through ``ridc_integrate_noalloc`` (no device allocation by the
    library; its fixed per-GPU array holds the rings).  ``nonfinite`` (optional): a cleared
    int32 CUDA tensor set to 1 when the result holds a NaN or Inf.  Asynchronous."""
    import torch
    if uT is None:
        uT = torch.empty_like(u0)
    p = make_problem(prob, dt)
    flag = None
    if nonfinite is not None:
        if not (nonfinite.is_cuda and nonfinite.dtype == torch.int32):
            raise TypeError("nonfinite must be an int32 CUDA tensor")
        flag = ctypes.c_void_p(nonfinite.data_ptr())
    _check(_lib.ridc_integrate_noalloc(ctypes.byref(p), _stream_ptr(stream), _ptr(u0),
                                       int(nsteps), _ptr(uT), flag))
    return uT


def tune_save(path: str | None = None):
    """Write the tuning table (measured launch shapes) to ``path`` (None: the default cache)."""
    _check(_lib.ridc_tune_save(path.encode() if path else None))


def tune_load(path: str | None = None):
    """Merge the launch shapes recorded in ``path`` (None: the default cache) into the table."""
    _check(_lib.ridc_tune_load(path.encode() if path else None))


def tune_clear():
    """Forget every recorded launch shape (the autotuners measure again)."""
    _check(_lib.ridc_tune_clear())


def pipeline_steps(nt: int, order: int) -> int:
    return nt + order * (order - 1) // 2 if nt > 0 else 0


def grid_h(prob: dict) -> float:
    n = int(prob["n"])
    return prob["length"] / n if prob["bc"] == "periodic" else prob["length"] / (n + 1)


__all__ = ["Ridc", "RidcError", "advance", "integrate_batch", "set_batch_tile", "autotune_batch",
           "batch_kernel_time", "integrate_noalloc", "make_ext", "uses_ext", "stage_weights",
           "tune_save", "tune_load", "tune_clear",
           "make_problem", "footprint_bytes",
           "quadrature_weights", "pcr_plan", "pipeline_steps", "library_path", "lib", "EXPORTED",
           "math"]
