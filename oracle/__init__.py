"""CPU float64 oracle (test infrastructure only; the library never imports it)."""
from .nys_oracle import *  # noqa: F401,F403
