"""Seeded synthetic inputs shared by the oracle-based tests and the GPU path.

This package holds random draws and memory layout only -- none of the method's
arithmetic -- so that the oracle and the HIP library can be fed identical inputs
without sharing any code that computes a result.
"""
from .workloads import *  # noqa: F401,F403
