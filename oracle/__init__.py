"""FP64 CPU oracle for RaBitQ; test infrastructure only (see rabitq_oracle)."""
from .rabitq_oracle import *  # noqa: F401,F403
