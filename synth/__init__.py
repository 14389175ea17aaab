"""Seeded synthetic point clouds for the flooding path.

This module only draws random geometry: it holds none of the flood
method's arithmetic, so both the GPU path and the CPU oracle can be fed
from it without sharing any computation.  Every generator returns
float32 arrays of shape [N, 3], row-major, and is fully determined by
its seed (numpy PCG64).

The paper's datasets (rhinovirus and coral scans, swisscheese, rocks,
corals, mcb-c, modelnet10) are not available; these surfaces stand in
for them: points uniform in area on spheres, tori and axis-aligned box
surfaces placed in the unit cube, plus isotropic Gaussian noise.
"""
from .clouds import (  # noqa: F401
    sphere_surface, torus_surface, box_surface, random_rotation,
    primitive_mix, config_cloud, batched_clouds, differentiable_clouds,
    circle_points, lattice_points, swisscheese, planar_cheese, CONFIGS,
)
