"""Seeded synthetic inputs shared by the tests, the bench and the oracle checks.

This module holds no arithmetic of the solver: it only draws right-hand sides
and initial data (sums of Gaussian bumps evaluated on the interior grid of a
box, random fields, domain masks), and the problem lists of the benchmark workloads.
"""
from .gen import (bump_field, grid_axis, l_shape_mask, learned_training_plan, octagon_mask, power_law_field, random_mask,
                  white_noise, workload_elliptic_64, workload_elliptic_1024, workload_rhs_256cubed, workload_uneven_steps)

__all__ = ["bump_field", "grid_axis", "workload_elliptic_64", "workload_elliptic_1024", "workload_rhs_256cubed",
           "workload_uneven_steps", "white_noise", "random_mask", "l_shape_mask", "octagon_mask", "power_law_field", "learned_training_plan"]
