"""Seeded synthetic workloads for IVF-RaBitQ search.

This package only draws random numbers: it holds no part of the search
method's arithmetic, so both the CPU oracle and the GPU library may take their
inputs from it without sharing any computation.
"""
from .workloads import WORKLOADS, Workload, get  # noqa: F401
from .gen import database, queries, arrivals  # noqa: F401
