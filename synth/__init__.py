"""Seeded synthetic inputs shared by the product, its tests and the benchmark.

This package holds geometry and random numbers only: closed surfaces given as
curved quadratic triangles (six geometric nodes each), random complex
densities and plane-wave directions, and random block data for the learned
preconditioner's loss.  It contains none of the method's
arithmetic (no quadrature rule, no kernel, no normal or weight computation);
both the HIP path and the oracle derive those on their own.
"""

from .meshes import (  # noqa: F401
    octa_sphere,
    ellipsoid,
    star_surface,
    n_for_dofs,
    random_densities,
    random_directions,
    instance_batch,
)
from .blocks import learned_blocks  # noqa: F401
