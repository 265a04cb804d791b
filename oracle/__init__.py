"""FP64 CPU oracle for the explicit interfacial system of the overlapping-circle
substructuring method (Moron-Vidal, Bernal, Suzuki, arXiv 2311.08946).

TEST INFRASTRUCTURE ONLY.  Nothing in the library or its Python binding may
import, call or execute this package; only the tests, the smoke check and the
benchmark's CPU-baseline leg do.  It shares no code with the HIP path: the two
meet only in the seeded workload descriptions of the top-level ``workloads``
module.

Every function is a plain, slow, readable restatement of the paper's
definitions in float64 (NumPy/SciPy), citing the section or equation it
follows:

* ``fields``      coefficient fields of the model problem (Section 2, eqs. 1-3)
* ``geometry``    cover, subdomains, interfaces, knots, stencils, row choice
                  (Section 2.1, eqs. 4-12; Section 3.2)
* ``cardinal``    Fourier and inverse-multiquadric cardinal functions
                  (Section 2.2, eqs. 13-22)
* ``spectral``    polar Chebyshev x Fourier collocation of the local problems
                  and the floating rows (Section 2.4 eqs. 31-35, Section 3.3
                  eqs. 40-41)
* ``philox``      the Philox4x32-10 counter-based generator (Salmon et al.,
                  SC'11), uniform and Box-Muller maps
* ``montecarlo``  Euler-Maruyama Feynman-Kac estimates for perimeter rows
                  (Section 2.3 eqs. 25-30, Appendix eq. 53), plain or with the
                  boundary-shifted scheme of the paper's ref. [15]
* ``assemble``    the sparse system C u = r (eqs. 28-30; averaged rows,
                  eqs. 38-39), its direct solve and diagnostics
* ``ras``         the one-level restricted additive Schwarz preconditioner and
                  right-preconditioned restarted GMRES (Section 4, eqs. 42-45)
* ``adjoint``     exact derivative of the discrete map with respect to the
                  node samples of the coefficients (not in the paper)

Functions whose result has no independent pin say "parity unpinned" in their
docstring.
"""
