"""Seeded synthetic input generators (no arithmetic of the method)."""
from .workloads import *  # noqa: F401,F403
