"""FP64 CPU oracle (test infrastructure only; see hopf_oracle's header)."""
from .hopf_oracle import *  # noqa: F401,F403
