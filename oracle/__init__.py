"""FP64 CPU oracle (test infrastructure only; see ``oracle.wm_oracle``)."""
from .wm_oracle import *  # noqa: F401,F403
