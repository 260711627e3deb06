"""FP64 CPU oracle of the DEC steady-diffusion path (TEST INFRASTRUCTURE ONLY).

Plain, slow, obviously-correct numpy/scipy code that states what the path
computes, written from the paper's Section 2 (primal/dual complexes, the
coboundary d, circumcentric diagonal Hodge stars, Dirichlet/Neumann data,
zero-conductivity cracks) and from textbook definitions (circumcentres,
conjugate gradients, factored sparse approximate inverse, iterative
refinement).  Only the test suite, the smoke entry point and the benchmark's
CPU-baseline leg may import it; the product library never does, and this
package imports nothing from the product library.

Temperature lives on the Delaunay vertices (a primal 0-form); the operator is
L = d0^T *1 d0 with *1 the diagonal circumcentric Hodge star on edges scaled
by a per-edge conductivity (Section 2.1, the exterior-calculus statement of
the Fourier law and conservation).  See each function for the passage it
follows.
"""
from .topology import (LOCAL_EDGES, edges_of, tet_edge_ids, faces_of, d0_matrix, d1_matrix,
                       check_mesh, vertex_degrees, boundary_faces)
from .geometry import (circumcenter_tet, circumcenter_tri, elementary_dual_areas, tet_volumes,
                       dual_areas, edge_lengths, hodge1, boundary_dual_areas, neumann_load, SNAP_REL)
from .cracks import crack_cut
from .laplacian import (assemble, isolated_components, apply_bc, lumped_vertex_volumes,
                        rms_error)
from .krylov import pcg, fsai_factor, fsai_pattern, iterative_refinement, PCGResult
from .flux import flux_effective_conductivity
from .cracking import (flux_density, max_flux_edge, CrackingSystem, cracking_process)
from . import dual
from .reorder import spatial_order

__all__ = [
    "LOCAL_EDGES", "edges_of", "tet_edge_ids", "faces_of", "d0_matrix", "d1_matrix",
    "check_mesh", "vertex_degrees", "boundary_faces",
    "circumcenter_tet", "circumcenter_tri", "elementary_dual_areas", "tet_volumes",
    "dual_areas", "edge_lengths", "hodge1", "boundary_dual_areas", "neumann_load", "SNAP_REL",
    "crack_cut",
    "assemble", "isolated_components", "apply_bc", "lumped_vertex_volumes", "rms_error",
    "pcg", "fsai_factor", "fsai_pattern", "iterative_refinement", "PCGResult",
    "flux_effective_conductivity",
    "flux_density", "max_flux_edge", "CrackingSystem", "cracking_process",
    "dual", "spatial_order",
]
