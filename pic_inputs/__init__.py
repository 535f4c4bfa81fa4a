"""Seeded synthetic inputs shared by the oracle and the HIP path.

This package holds only data: workload descriptions (geometry rectangles,
circuit element values, gas, particle counts, time step) and seeded random
particle sets.  It contains none of the method's arithmetic: no deposit, push,
collision, field-solve or circuit code.  Both the CPU oracle and the GPU
binding import it; neither imports the other.
"""
from .workloads import WORKLOADS, workload, gec_geometry, parallel_plate_geometry  # noqa: F401
from .particles import random_particles  # noqa: F401
