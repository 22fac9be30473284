"""Seeded input generators (grids, matrices, symmetry maps, right-hand sides)."""
from .problems import (make_problem, config_problem, batch_problems, transmissibility,  # noqa: F401
                       base_blocks, assemble_full, tanh_nodes, Problem, BaseFaces,
                       FACE_INTERIOR, FACE_DIRICHLET, FACE_MIRROR, CONFIG_SEED0,
                       make_repeated_problem, CopiesProblem)
