"""MI355X (gfx950) semi-implicit RIDC: HIP kernels behind a C ABI, with a thin Python binding.

``paper_1209_4297_amd.ridc`` loads ``libridc.so`` (built in-tree by ``build.py``) and fails
loudly when it is missing; there is no CPU fallback.
"""
import os

PKG_DIR = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG_DIR, "libridc.so")

__all__ = ["PKG_DIR", "LIB_PATH"]
