"""Schoolbook polynomial products (Background, polynomial multiplication using NTT).

The paper writes the schoolbook product of two polynomials as
sum_j (sum_{i<=j} a_i b_(j-i) mod q) x^j, an O(n^2) sum.  The fused pipeline
NTT(a), NTT(b) -> point-wise mulmod -> INTT computes the product in the ring
Z_q[X]/(X^N + 1); the oracle therefore takes the schoolbook product and wraps
it with X^N = -1 (reading: negacyclic reduction of the paper's product):

    c_k = sum_{i+j=k} a_i b_j - sum_{i+j=k+N} a_i b_j   (mod q).
"""
from typing import Iterable, List, Sequence

from .modarith import check_canonical


def schoolbook(a: Sequence[int], b: Sequence[int], q: int) -> List[int]:
    """Full product of degree < len(a)+len(b)-1, coefficients reduced mod q."""
    check_canonical(a, q); check_canonical(b, q)
    out = [0] * (len(a) + len(b) - 1)
    for i, ai in enumerate(a):
        for j, bj in enumerate(b):
            out[i + j] += ai * bj
    return [c % q for c in out]


def negacyclic(a: Sequence[int], b: Sequence[int], q: int) -> List[int]:
    """Product modulo X^N + 1, from the schoolbook product."""
    n = len(a)
    if len(b) != n:
        raise ValueError("length mismatch")
    full = schoolbook(a, b, q)
    out = full[:n] + [0] * (n - len(full[:n]))
    for k in range(n, len(full)):
        out[k - n] -= full[k]            # X^k = -X^(k-N)
    return [c % q for c in out]


def negacyclic_at(a: Sequence[int], b: Sequence[int], q: int, ks: Iterable[int]) -> List[int]:
    """Selected coefficients of the negacyclic product, O(N) each."""
    n = len(a)
    out = []
    for k in ks:
        acc = 0
        for i in range(n):
            j = k - i
            if j >= 0:
                acc += a[i] * b[j]
            else:
                acc -= a[i] * b[j + n]
        out.append(acc % q)
    return out
