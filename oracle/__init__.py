"""FP64 CPU oracle for the implicit filter -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct NumPy/SciPy implementation of what the
filter computes, written from the paper's equations. It is the reference
that the HIP library is checked against; the product path never imports
it. Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` may import, call or execute anything in this package.

It shares no code with the library (``paper_2404_07398_amd``): both consume
the seeded inputs of ``workloads`` and nothing else.

Contents
--------
operators : active cells / dofs, flat-facet geometry, cotangent stiffness
            (Galerkin P1 form of Sect. 2.1.1), the finite-volume median-dual
            route (same section), lumped mass, order-n operator (Eq. 5 and
            the biharmonic FE form), the cell-vector operator (Eq. 7), the
            vertex FE vector Laplacian with metric terms (Sect. 2.1.2).
solve     : the system ``S = M + gamma/k^(2n) K_n`` (Eq. 1 with Eq. 4/5),
            dense Cholesky for small meshes, Jacobi-PCG from ``x0 = phi``
            (residual form of Sect. 2.2.2) with extended-precision
            refinement for larger ones.
spectrum  : filtered-energy spectrum (coarse-graining, Sect. 2.1) and its
            finite-difference density.

Every function names the passage it follows. Functions without a pin say
"parity unpinned" in their docstring.
"""
from .operators import (
    CellScalarOperator,
    ScalarOperator,
    VectorOperator,
    VertexVectorOperator,
    active_cells,
    circumcenter_operator,
    scalar_operator,
    vector_operator,
    vertex_vector_operator,
    voronoi_operator,
    cot_stiffness,
    fv_stiffness,
    lumped_mass,
    order_n,
)
from .solve import (
    system_matrix,
    filter_scalar,
    filter_vector,
    filter_vertex_vector,
    project_cells_to_vertices,
    filter_dense,
    pcg_jacobi,
    refine_solve,
    to_dofs,
    from_dofs,
)
from .spectrum import discrete_symbol, energy, fig8_modes, filtered_energy_of_modes, spectrum_density

__all__ = [
    "ScalarOperator",
    "VectorOperator",
    "VertexVectorOperator",
    "vertex_vector_operator",
    "filter_vertex_vector",
    "project_cells_to_vertices",
    "active_cells",
    "scalar_operator",
    "vector_operator",
    "voronoi_operator",
    "circumcenter_operator",
    "CellScalarOperator",
    "cot_stiffness",
    "fv_stiffness",
    "lumped_mass",
    "order_n",
    "system_matrix",
    "filter_scalar",
    "filter_vector",
    "filter_dense",
    "pcg_jacobi",
    "refine_solve",
    "to_dofs",
    "from_dofs",
    "energy",
    "spectrum_density",
    "discrete_symbol",
    "filtered_energy_of_modes",
    "fig8_modes",
]
