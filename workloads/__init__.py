"""Seeded synthetic problem generators shared by the tests, the benchmark and
the smoke check.

This package describes *problems* only: the uniform computational grid, the
coordinate map onto the physical domain (node coordinates and, where the map
is analytic, its closed-form partial derivatives), the physical charge density
sampled at the mapped nodes, the interior Dirichlet mask and the Dirichlet
data.  It holds none of the solver's arithmetic (no Jacobian-to-permittivity
transform, no stencil, no multigrid); both the CPU oracle and the GPU library
take these arrays as inputs.
"""

from .gen import (  # noqa: F401
    GridProblem,
    identity_map,
    affine_map,
    sinusoidal_map,
    manufactured_sinusoidal,
    perturbed_circle,
    polar_semi_annulus,
    sinh_stretch,
    square_to_disc,
    disc_boundary,
    disc_on_grid,
    embedded_body_boundary,
    embedded_flow,
    gaussian_sources,
    random_sinusoidal,
    batch_mixed,
    serving_stream,
    draw_annulus_sources,
)
