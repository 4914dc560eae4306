"""Seeded synthetic input scenes (no solver arithmetic)."""
from .scenes import *  # noqa: F401,F403
