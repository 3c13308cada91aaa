"""Seeded synthetic inputs (meshes, cell suspensions, forces) shared by the
oracle, the tests and the benchmark. Holds no solver arithmetic."""
from . import meshes, suspensions  # noqa: F401
