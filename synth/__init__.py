"""Seeded synthetic inputs for DEANN's query path.

This module only draws random numbers and lays them out as float32 arrays.  It
holds none of the method's arithmetic (no distances, kernels, neighbour search
or sampling): both the FP64 oracle and the HIP path receive the same bytes from
here and nothing else is shared between them.
"""
from .mixtures import (  # noqa: F401
    MixtureSpec, WORKLOADS, make_mixture, workload, query_subset,
)
