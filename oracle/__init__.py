"""FP64 CPU oracle (test infrastructure only; see pty_oracle's header)."""
from .pty_oracle import *  # noqa: F401,F403
from .pty_oracle import Geometry, LOSS_KINDS  # noqa: F401
