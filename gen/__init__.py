"""Seeded synthetic inputs: structured Kuhn-tetrahedra cube meshes, P1 finite element
assembly (linear elasticity and Poisson) into block CSR, Dirichlet masks and random
right-hand sides.

This package produces the *problem* (the matrix A of the paper's problem statement,
section "fem": Problems prob:gg and prob:epseps) and holds none of the multigrid
method's arithmetic.  Both the CPU oracle and the GPU library consume its output.
"""
from .kuhn import (  # noqa: F401
    KuhnProblem,
    kuhn_mesh,
    assemble_elasticity,
    assemble_poisson,
    make_problem,
    lame_from_young,
    sphere_inclusions,
    WORKLOADS,
)
