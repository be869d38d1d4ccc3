"""Seeded synthetic inputs (meshes, surfaces, poses) shared by the oracle tests,
the HIP-path tests and the benchmark.  Holds no step of the method."""
from . import meshes, configs  # noqa: F401
