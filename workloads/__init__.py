"""Seeded synthetic inputs shared by the HIP path and the CPU oracle.

This package holds no charge-transport arithmetic: it only draws the
event-level quantities (photon energy, absorption depth, entry point,
track geometry) and states the sensor settings of each named workload.
Both the library binding and the oracle binding consume the same objects.
"""
from .events import (  # noqa: F401
    Sensor,
    Batch,
    WORKLOADS,
    make_workload,
    single_8kev,
    batch_8kev, batch_8kev_eh,
    mixed_energy,
    gamma_60kev,
    track_200kev,
    track_walks,
    explicit_batch,
    GenParams,
    generator_25kev,
)
