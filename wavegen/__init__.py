"""Seeded synthetic inputs (meshes, initial volume fractions, face fluxes, velocities).

This package serves both the CPU oracle and the GPU library as a source of
inputs only; it contains none of the advection method's arithmetic.
"""
from .mesh import (PATCH_CYCLIC, PATCH_EMPTY, PATCH_INOUT, PATCH_WALL, Mesh, Patch, graded_halves,
                   hex_block)
from .fields import (AiryWave, UniformPlusTaylorGreen, alpha_column_plus_wave_3d, alpha_cosine_2d, dynamic_pressure,
                     cell_fraction_below_cosine, courant_dt, fluxes_from_edge_integral)
from .poly import (PolyWorkload, alpha_sampled, cell_geometry, fluxes_from_potential, mesh_from_cells, poly_airy,
                   merged_block, mixed_block, poly_violent, prism_block, pyramid_block, tet_block)
from .configs import (Workload, adjoint_case, airy_1024x256, airy_ensemble, airy_slab, cosine_uniform, perturbed_box,
                      slab_mesh, violent_3d)

__all__ = [n for n in dir() if not n.startswith("_")]
