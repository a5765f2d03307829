"""FP64 CPU oracle (test infrastructure only; see qfdtd_oracle)."""
from .qfdtd_oracle import *  # noqa: F401,F403
