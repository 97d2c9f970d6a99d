"""Modular arithmetic by definition (Background, modular arithmetic).

The paper defines c = a + b, a - b and a*b modulo q for a, b, c in Z_q, and
captures point-wise polynomial operations as BLAS: vector add, vector sub,
point-wise vector mul and axpy y = a*x + y (Background, polynomial operations).
The fast algorithms of the paper (conditional subtraction, Eq. saddmod; 
conditional addition, Eq. ssubmod; Barrett reduction, Eq. barrett) all return
the unique canonical residue in [0, q); this oracle computes that residue with
Python's exact ``%``.  Inputs must already be canonical (0 <= a, b < q), as the
paper assumes; ``check_canonical`` enforces it.

Parity pins: tests/test_oracle.py (special cases, inverse identities,
Fermat's little theorem, brute force over all pairs for a tiny modulus).
"""
from typing import List, Sequence


def check_canonical(xs: Sequence[int], q: int) -> None:
    for x in xs:
        if not 0 <= x < q:
            raise ValueError("input residue outside [0, q)")


def addmod(a: int, b: int, q: int) -> int:
    return (a + b) % q


def submod(a: int, b: int, q: int) -> int:
    return (a - b) % q


def mulmod(a: int, b: int, q: int) -> int:
    return (a * b) % q


def vec_addmod(a: Sequence[int], b: Sequence[int], q: int) -> List[int]:
    check_canonical(a, q); check_canonical(b, q)
    if len(a) != len(b):
        raise ValueError("length mismatch")
    return [addmod(x, y, q) for x, y in zip(a, b)]


def vec_submod(a: Sequence[int], b: Sequence[int], q: int) -> List[int]:
    check_canonical(a, q); check_canonical(b, q)
    if len(a) != len(b):
        raise ValueError("length mismatch")
    return [submod(x, y, q) for x, y in zip(a, b)]


def vec_mulmod(a: Sequence[int], b: Sequence[int], q: int) -> List[int]:
    check_canonical(a, q); check_canonical(b, q)
    if len(a) != len(b):
        raise ValueError("length mismatch")
    return [mulmod(x, y, q) for x, y in zip(a, b)]


def vec_axpymod(alpha: int, x: Sequence[int], y: Sequence[int], q: int) -> List[int]:
    """y <- alpha*x + y (mod q), the BLAS level-1 axpy over Z_q."""
    check_canonical([alpha], q); check_canonical(x, q); check_canonical(y, q)
    if len(x) != len(y):
        raise ValueError("length mismatch")
    return [(alpha * xi + yi) % q for xi, yi in zip(x, y)]
