"""Seeded synthetic workloads (systems and query points); no solver arithmetic."""
from .workloads import (SystemSpec, double_integrator, random_system,  # noqa: F401
                        uniform_box_points, gaussian_points,
                        tychastic_double_integrator, tychastic_points,
                        unscented_weights, unscented_double_integrator, unscented_points)
