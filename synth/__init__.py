"""Seeded synthetic inputs (no registration arithmetic); shared by tests and bench."""
from .generators import *  # noqa: F401,F403
