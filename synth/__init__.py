"""Seeded synthetic inputs shared by tests, the benchmark and the smoke check."""
from .stacks import WORKLOADS, Workload, crop, land_cover, make_sequence, make_stack, smooth_field, true_phase  # noqa: F401
