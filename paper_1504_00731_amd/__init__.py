"""MI355X-native WENO-theta library (adaptive WENO-theta finite differences, HIP/gfx950)."""
from . import workloads  # noqa: F401
