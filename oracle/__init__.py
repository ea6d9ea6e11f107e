"""Reference CPU implementation of the pseudo-flow solvers (test infrastructure only)."""
from .pseudoflow_oracle import *  # noqa: F401,F403
