"""Plain, slow FP64 CPU oracle for the T-REXI shallow-water hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import or call anything in this package.
The product (the HIP library and its Python binding) never does, and this
package never imports the product.  It shares no code with the GPU path; the
only common module is ``synth`` (seeded inputs, none of the method's
arithmetic).

Contents, each written from the paper (Schreiber & Loft, "A Parallel
Time-Integrator for Solving the Linearized Shallow Water Equations on the
Rotating Sphere"):

* ``coeffs``   - REXI coefficients: Gaussian rational fit, Gaussian sum for
                 e^{ix}, two-sided merge, beta renormalisation (Sections 4.1, 6.1).
* ``sh``       - Gauss-Legendre grid, orthonormal associated Legendre functions,
                 plain DFT + quadrature analysis and direct synthesis (Section 3).
* ``operator`` - the linear SWE operator (Eq. (1)) in spherical-harmonic space,
                 one dense block per zonal order m, in energy-scaled variables.
* ``rexi``     - one T-REXI step as the literal sum over 2N shifted banded
                 solves (Section 4.2, Algorithm 1's loop-and-reduce), its
                 adjoint, and multi-step driving.

Pinned by ``tests/test_oracle_*.py``.  Nothing here is "parity unpinned".
"""
