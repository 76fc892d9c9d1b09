"""CPU oracle for the POLFED hot path (Sierant, Lewenstein, Zakrzewski,
arXiv:2005.09534).

THIS PACKAGE IS TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the test
suite (``tests/``), ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import or run it.  The GPU library never calls it, links it or
falls back to it, and it shares no code, table or constant with the HIP path.

Everything here is plain, slow and FP64 (NumPy / SciPy), written so that a
reader can hold it against the paper:

* ``chain``     -- the spin chain of eq. (XXZ): Sz=0 basis, ranking, CSR H.
* ``chebyshev`` -- the polynomial spectral transformation eq. (polyTransf):
  coefficients c_n, normalisation D, the filter applied by the plain forward
  three-term recurrence, the Gaussian density of states and the order rule
  n_P(K) = N_ev (main text "POLFED algorithm", Supplement "Convergence").
* ``lanczos``   -- spectral bounds, block Lanczos with full
  reorthogonalisation eqs. (Lan1)-(Lan2), Ritz extraction, Rayleigh-Ritz and
  residuals: the full POLFED solve.
* ``observables`` -- entanglement entropy of eigenvectors over the half-ring
  cuts and the mean gap ratio of eigenvalues (main text, "Entanglement
  entropy and level statistics").
* ``kpm``       -- the density of states by the kernel polynomial method
  (Chebyshev moments from random vectors, Jackson damping, the count of
  states in the filter's main lobe and the order rule built on it).
* ``dense``     -- the definition of the answer: the N_ev eigenpairs of H
  nearest the target, by dense diagonalisation (or a library shift-invert
  eigensolver where dense is too large).

Parity status of each function is stated in its docstring.  Every function is
pinned by a test in ``tests/test_oracle_pins.py`` against something other than
itself (brute force, a Kronecker-product construction, closed forms, free
fermions, dense diagonalisation, invariants).
"""

from . import chain, chebyshev, lanczos, dense, observables, kpm  # noqa: F401
