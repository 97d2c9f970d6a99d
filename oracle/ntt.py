"""Number theoretic transforms by definition.

Eq. (ntt) defines the n-point transform y_k = sum_j x_j * omega^(jk) mod q
with omega a primitive n-th root of unity (Background, polynomial
multiplication using NTT).  ``ntt_cyclic`` writes exactly that sum out.

Readings taken where the paper is silent:

1. Negacyclic form.  The workload is the negacyclic transform over
   Z_q[X]/(X^N + 1): A_k = sum_j a_j psi^(j(2k+1)), psi a primitive 2N-th
   root.  It is Eq. (ntt) applied to the twisted input x_j = a_j psi^j with
   omega_N = psi^2, and is computed that way here (``ntt_negacyclic``).
2. Root.  psi is the canonical (smallest) primitive 2N-th root
   (``roots.canonical_psi``) unless the caller passes one.
3. Order.  Inputs and outputs are in natural order (index k holds A_k).
4. Inverse.  The paper never defines it; the oracle uses the exact inverse
   a_j = N^-1 psi^-j sum_k A_k psi^(-2jk), i.e. Eq. (ntt) with omega_N^-1
   followed by the untwist and the 1/N scale, so that INTT(NTT(a)) = a.
5. Length.  A polynomial has N coefficients (degree < N), matching "n-point"
   in Eq. (ntt).

Cost: ``ntt_cyclic`` is O(N^2) exact integer work (one reduction per output);
use it for N up to a few thousand.  For large N, ``forward_at`` and
``inverse_at`` evaluate single output indices from the same definitions in
O(N) each.
"""
from typing import Iterable, List, Optional, Sequence

from . import roots
from .modarith import check_canonical


def ntt_cyclic(x: Sequence[int], omega: int, q: int) -> List[int]:
    """Eq. (ntt): y_k = sum_{j<n} x_j omega^(jk) mod q, 0 <= k < n."""
    n = len(x)
    # omega^n = 1, so omega^(jk) = omega^(jk mod n); tabulate omega^e once.
    pw = [1] * n
    for e in range(1, n):
        pw[e] = pw[e - 1] * omega % q
    out = []
    for k in range(n):
        acc = 0
        for j in range(n):
            acc += x[j] * pw[(j * k) % n]
        out.append(acc % q)
    return out


def _root(q: int, n: int, psi: Optional[int]) -> int:
    roots.check_ntt_modulus(q, n)
    if psi is None:
        return roots.canonical_psi(q, n)
    if pow(psi, n, q) != q - 1:
        raise ValueError("psi is not a primitive 2N-th root of unity")
    return psi


def ntt_negacyclic(a: Sequence[int], q: int, psi: Optional[int] = None) -> List[int]:
    """Forward negacyclic NTT, natural order: A_k = sum_j a_j psi^(j(2k+1)) mod q."""
    n = len(a)
    check_canonical(a, q)
    psi = _root(q, n, psi)
    twisted = []
    t = 1
    for j in range(n):
        twisted.append(a[j] * t % q)    # x_j = a_j psi^j
        t = t * psi % q
    return ntt_cyclic(twisted, psi * psi % q, q)


def intt_negacyclic(A: Sequence[int], q: int, psi: Optional[int] = None) -> List[int]:
    """Inverse negacyclic NTT: a_j = N^-1 psi^-j sum_k A_k psi^(-2jk) mod q."""
    n = len(A)
    check_canonical(A, q)
    psi = _root(q, n, psi)
    psi_inv = pow(psi, -1, q)
    n_inv = pow(n, -1, q)
    y = ntt_cyclic(A, psi_inv * psi_inv % q, q)
    out = []
    t = 1
    for j in range(n):
        out.append(y[j] * t % q * n_inv % q)   # untwist psi^-j, scale N^-1
        t = t * psi_inv % q
    return out


def forward_at(a: Sequence[int], q: int, ks: Iterable[int], psi: Optional[int] = None) -> List[int]:
    """A_k for selected k, straight from the definition (O(N) per index)."""
    n = len(a)
    psi = _root(q, n, psi)
    out = []
    for k in ks:
        e = pow(psi, 2 * k + 1, q)      # A_k = sum_j a_j (psi^(2k+1))^j
        acc, p = 0, 1
        for j in range(n):
            acc += a[j] * p
            p = p * e % q
        out.append(acc % q)
    return out


def inverse_at(A: Sequence[int], q: int, js: Iterable[int], psi: Optional[int] = None) -> List[int]:
    """a_j for selected j, straight from the inverse definition (O(N) per index)."""
    n = len(A)
    psi = _root(q, n, psi)
    psi_inv = pow(psi, -1, q)
    n_inv = pow(n, -1, q)
    out = []
    for j in js:
        e = pow(psi_inv, 2 * j, q)      # psi^(-2jk) = e^k
        acc, p = 0, 1
        for k in range(n):
            acc += A[k] * p
            p = p * e % q
        out.append(acc % q * pow(psi_inv, j, q) % q * n_inv % q)
    return out
