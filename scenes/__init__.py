"""Seeded synthetic inputs (point clouds, features, poses, frame-pair graphs)."""
from .synth import *  # noqa: F401,F403
from .synth import __all__  # noqa: F401
