"""FP64 CPU oracle for semi-implicit RIDC (test infrastructure only; see ``ridc_oracle``)."""
from .ridc_oracle import *  # noqa: F401,F403
