"""CPU oracle for the solid Newton step — TEST INFRASTRUCTURE ONLY.

A plain, slow, fp64 implementation of what the GPU path computes, written
from the paper (Langer & Yang, "Numerical simulation of fluid-structure
interaction problems with hyperelastic models I: a partitioned approach"):

* ``fe``      element kinematics, the two material laws, the stabilised
              P1-P1 residual and consistent tangent, global assembly,
              Dirichlet elimination, the blocks A, B2 and the Schur diagonal;
* ``rng``     the counter-based SplitMix64 generator used for PMIS weights;
* ``amg``     strength, PMIS, modified classical interpolation, Galerkin RAP,
              smoothers, coarsest LU, V-cycle, convergence-factor judge;
* ``krylov``  the block-triangular preconditioner and FGMRES;
* ``newton``  the Newton loop with the mass-norm stopping rule;
* ``mlp``     the learned-interpolation network: features, forward,
              backward, loss and the local ideal-interpolation target;
* ``newmark`` the Newmark-beta update of the structure;
* ``vanka``   the coupled (u, p) AMG with the Vanka smoother;
* ``fluid``   the stabilised P1-P1 fluid step on a moving mesh and the
              harmonic mesh extension;
* ``fsi``     the Dirichlet-Neumann iteration with Aitken relaxation.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it.  It shares no code with the HIP library and
must never be used as a fallback for it.
"""
