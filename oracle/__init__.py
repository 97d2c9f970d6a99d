"""CPU oracle for the multi-word modular NTT / BLAS path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package; the library never
calls it, and nothing here is shared with the HIP kernels.

Everything is written from the paper's definitions in plain Python integers
(exact, arbitrary width), slow and obviously correct:

* ``modarith`` -- modular add / sub / mul and axpy (Background, modular
  arithmetic; polynomial operations as BLAS).
* ``roots``    -- the canonical primitive 2N-th root of unity.
* ``ntt``      -- the n-point transform of Eq. (ntt) by its definition, the
  negacyclic forward / inverse transforms built on it, and per-index
  evaluations for large N.
* ``polymul``  -- schoolbook polynomial products (Background, polynomial
  multiplication using NTT), reduced modulo X^N + 1.

Readings of the paper that the oracle takes where the text is silent
(negacyclic twist, choice of root, inverse scaling, output order) are listed in
each module's docstring.

Pins: ``tests/oracle_pins.py`` (run by ``tests/test_oracle.py``) checks every
function here against the paper's worked example, closed forms, brute force on
small moduli and independent evaluations, at small and at 60-, 124- and 252-bit
primes; ``tests/test_oracle_mutations.py`` plants plausible mistakes in this
package and checks that each one fails a pin.
"""
from . import modarith, roots, ntt, polymul  # noqa: F401
