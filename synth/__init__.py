"""Seeded synthetic problem generators shared by the oracle, the tests and the
benchmark.  Holds no multigrid arithmetic."""
from .problems import *  # noqa: F401,F403
