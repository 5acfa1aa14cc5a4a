"""FP64 CPU oracle (test infrastructure only; see sgn_oracle's header)."""
from .sgn_oracle import *  # noqa: F401,F403
