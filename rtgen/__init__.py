"""Seeded synthetic inputs (scenes, launched rays) shared by the GPU path and
its CPU checker; holds no part of the tracing or BVH arithmetic."""
from . import icosphere, scenes, workloads  # noqa: F401
