"""FP64 CPU oracle (test infrastructure only; see morlet_oracle)."""
from . import morlet_oracle  # noqa: F401
