"""Seeded synthetic workloads (configs and input generators) for tests and benchmarks."""
from . import configs, generate  # noqa: F401
