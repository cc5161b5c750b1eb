"""Seeded synthetic input generators (shared by the oracle and the GPU path)."""
from .synth import *  # noqa: F401,F403
