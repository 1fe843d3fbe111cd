"""Seeded synthetic workloads shared by tests and benchmark (inputs only)."""
from .synthetic import (CONFIGS, Config, Workload, batch_configs, random_problem, stored_values,  # noqa: F401
                        to_storage)
