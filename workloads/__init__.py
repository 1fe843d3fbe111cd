"""Seeded synthetic workloads shared by tests and benchmark (inputs only)."""
from .synthetic import CONFIGS, Config, Workload, random_problem, stored_values, to_storage  # noqa: F401
