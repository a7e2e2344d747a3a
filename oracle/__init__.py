"""Plain FP64 CPU oracle for the differentiable direct N-body method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, calls or
links anything in this directory; only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark script do.  The oracle shares no code with the
HIP path: it has its own constants, its own force, potential, integrator,
adjoint and loss code, written from the textbook definitions that the paper
(arXiv 2511.22468, "Odisseo") names without printing.

Every function is written to be generic over the array dtype so that the same
code runs in float64, longdouble (brute-force pins) and complex128
(complex-step derivatives).  For that reason no function calls ``abs`` or
``np.linalg.norm`` on a differentiated quantity, and branches test only real
parts.

Modules
-------
constants  units and default potential parameters
forces     softened pair sum, NFW halo, Miyamoto-Nagai disk, energies
integrate  kick-drift-kick (Velocity-Verlet) integrator
mmd        Gaussian-kernel maximum mean discrepancy and its gradient
adjoint    discrete adjoint of the integrator (exact gradient of the map)
pipeline   back-integration of the progenitor, IC assembly, forward model
surrogate  orbit-frame density grid and the 4-256-256-256-2048 surrogate network
           with BF16 emulation, GELU, MSE and Adam
orbitfit   orbit-aligned frame, track observables, chi^2, its Hessian and
           Levenberg-Marquardt

Parity unpinned: absolute energy-drift levels and stream morphology have no
value in the paper to compare against (its figures are not available), so
they are reported, not pinned.
"""
