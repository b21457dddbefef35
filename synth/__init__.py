"""Seeded synthetic GNSS IF snapshots shared by tests and benchmarks.

Holds only signal synthesis (planted satellites, noise, quantisers).  It does
no acquisition arithmetic; the C/A chip sequences of planted satellites are
passed in by the caller.
"""
from .generator import *  # noqa: F401,F403
