"""Seeded synthetic graph and query generators (inputs only; no search arithmetic)."""
from .graphs import *  # noqa: F401,F403
from .graphs import Graph  # noqa: F401
