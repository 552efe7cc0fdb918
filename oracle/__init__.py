"""FP64 CPU oracle (test infrastructure only; see isam_oracle)."""
from .isam_oracle import *  # noqa: F401,F403
from .isam_oracle import Grids, FistaResult  # noqa: F401
