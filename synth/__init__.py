"""Seeded synthetic inputs (workload records, scanner LOR layout, phantoms, data).

Serves both the oracle-based tests and the GPU path; holds no reconstruction
arithmetic (no projector, no prior, no update rule).
"""

from . import configs, scanner  # noqa: F401
