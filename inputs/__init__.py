"""Seeded synthetic inputs shared by tests, benchmark and smoke check.

Nothing here computes any part of the tree force; see ``inputs.ic`` for the
cluster models and ``inputs.workloads`` for the named workload presets.
"""
from .ic import Cluster, plummer, king, salpeter_masses, king_scale  # noqa: F401
from .workloads import WORKLOADS, Workload, make_cluster  # noqa: F401
