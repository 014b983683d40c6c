"""Plain FP64 CPU oracle for the aMFP-BTE hot path.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and the
benchmark's CPU-baseline leg may import anything from this package; the GPU
library never does, and this package never imports the GPU library.  The two
share no code: the only common module is ``inputs.gen`` (seeded input
generators that contain none of the method's arithmetic).

What it computes (paper: section "Model", section "Implementation",
Algorithm 1, Appendix A "The aMFP-BTE", Appendix B "Heat conduction
equation"): the fixed point of the discrete coupled system

  sigma_i (T_iml - T_L,i) + Lambda_m (A_l T_ml)_i
        = Lambda_m [periodic-jump inflow + wall inflow from T_w]_il

with T_L = sum_ml D_ml T_ml (energy conservation) and diffuse wall
temperatures T_w (thermalising walls), found by the source iteration of
Eq. (iter) with the Fourier first guess of Eq. (fourier_iter), one sparse LU
factorisation per (MFP, direction) system reused across passes as the paper
does.  Also: the dense brute-force solve of the whole coupled system for tiny
meshes, kappa definitions, and the adjoint d kappa / d sigma.

Modules: material (row a1), mesh (a2), fourier (a3), bte (a4-a8), adjoint (a9),
umesh (unstructured 2D meshes: the upwind operator from general face vectors
and the heat-conduction first guess with the explicit non-orthogonal
correction of Appendix B).
"""
from .material import Material, material_weights, wall_weights
from .mesh import Mesh
from .fourier import fourier_solve
from .bte import Problem, source_iteration, dense_solve, kappa_cc, kappa_face, flux_map
from .adjoint import adjoint_source_iteration, adjoint_dense, gradient_from

__all__ = [
    "Material", "material_weights", "wall_weights", "Mesh", "fourier_solve",
    "Problem", "source_iteration", "dense_solve", "kappa_cc", "kappa_face", "flux_map",
    "adjoint_source_iteration", "adjoint_dense", "gradient_from",
]
from .umesh import UMesh, UProblem, fourier_nonorth, upwind_operator_u, dense_solve_u
