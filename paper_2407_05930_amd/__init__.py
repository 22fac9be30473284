"""Mirror-symmetric Poisson solver for AMD MI355X (gfx950).

Python front end of ``libmsp.so``: setup from a symmetric sparse matrix and
its symmetry map, then solve with the HIP path (Alg. 1 of arXiv 2407.05930
with the shared multigrid-reduction preconditioner).
"""
from .solver import BatchSolver, Solver, default_opts, make_opts  # noqa: F401
from ._lib import MspError  # noqa: F401
