"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds no arithmetic of the solver itself: it only draws gauge
fields, gauge transformations, sources and random starting vectors from
seeded generators, and lists the workload shapes.  Both the CPU oracle and
the HIP path receive the arrays it produces as plain inputs.
"""
from .gen import (su3_field, su3_random, gauss_spinor, point_sources,
                  gauss_vectors, lattice_volume)
from .configs import CONFIGS, get_config

__all__ = ["su3_field", "su3_random", "gauss_spinor", "point_sources",
           "gauss_vectors", "lattice_volume", "CONFIGS", "get_config"]
