"""Seeded synthetic workload generators.

This package only draws random numbers and lays out fixed workload constants.
It holds none of the interior-point method's arithmetic and none of the model
equations, so both the CPU oracle and the HIP path can take their inputs from it.
"""
from .generators import (  # noqa: F401
    DistillationWorkload,
    distillation_workload,
    batch_distillation_workloads,
    PlateWorkload,
    plate_workload,
    RefluxWorkload,
    reflux_workload,
    random_lq,
    PlateCaseWorkload,
    plate_case_workload,
    WORKLOADS,
)
