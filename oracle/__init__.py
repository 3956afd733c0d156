"""CPU FP64 oracle for the scale-resolved Li-S DG hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call,
link or execute this package: only the tests, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP path
(no kernels, headers, helpers, constant tables or pre/post-processing); the
only common dependency is the seeded input module ``synth``.

What it computes, in the paper's order and notation (arXiv 2511.05233):

* model.py       -- constants and parameters (Tab. 5), the Tradeoff
                    Chemistry stoichiometry (Tab. 3), the analytical
                    equilibrium initial state (Tab. InitialState), the 3D
                    localisation (Eq. 57) and the applied current (App. C).
* chem.py        -- pointwise constitutive laws: viscosity / Stokes-Einstein
                    (Eq. 02-03), Bruggeman (Sec. 2.3), the anion-eliminated
                    charge coefficients (Tab. 4), the specific surface
                    (Eq. 18), Butler-Volmer rates (Eq. 19-24), the smoothed
                    Heaviside regularisation (Eq. 56).
* dg.py          -- the interior-penalty DG residual (Eq. 43-47) on
                    tensor-product hexahedra, written as plain quadrature
                    sums, and its Jacobian-vector product by complex-step
                    differentiation.
* solve.py       -- element-diagonal Jacobian blocks, the backward-Euler
                    step (Eq. 50) solved by Newton, and the steady potential
                    initialisation.
* controllers.py -- the naive feedback controller and the H211b controller
                    with step doubling and Richardson extrapolation
                    (Eq. 51-54).
* outputs.py     -- cell voltage, volume means (Eq. A1-A3) and the discrete
                    conservation invariants.
* multigrid.py   -- the multilevel aggregation preconditioner of the Krylov
                    system (the GPU stand-in for the algebraic multigrid of
                    Sec. 2.9): Galerkin operators on nested voxel aggregates,
                    damped block-Jacobi smoothing, the V-cycle.

Every function is written to accept complex input where it can be reached
by a complex-step derivative: comparisons look at real parts only.
"""
