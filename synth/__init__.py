"""Seeded synthetic inputs shared by the tests and the benchmark (no reconstruction arithmetic)."""
from .generators import *  # noqa: F401,F403
