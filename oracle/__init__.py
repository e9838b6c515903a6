"""FP64 CPU oracle (test infrastructure; see plink_oracle's header)."""
from .plink_oracle import *  # noqa: F401,F403
from . import plink_oracle  # noqa: F401
