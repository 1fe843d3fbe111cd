"""Seeded synthetic workloads shared by tests and benchmark (inputs only)."""
from .synthetic import CONFIGS, Config, Workload, random_problem  # noqa: F401
