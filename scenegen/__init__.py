"""Seeded synthetic input scenes (no solver arithmetic)."""
from .scenes import *  # noqa: F401,F403
from .composites import CompositeScene, composite_cluster, composite_gas, composites, from_spheres  # noqa: F401
