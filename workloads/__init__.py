"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

Only problem data lives here (permeability fields, the EDFM fine-scale system,
fracture geometry, right-hand sides).  Nothing in this package implements any
step of the multiscale solver.
"""
from .edfm import FracturedSystem, Plate, Well, add_wells, build_system, lnk_field  # noqa: F401
from .configs import make_config, make_small, CONFIGS  # noqa: F401
