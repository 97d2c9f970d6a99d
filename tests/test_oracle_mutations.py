"""Plant plausible mistakes in the oracle (on the CPU) and check the pins catch each one.

A pin set that a dropped term, a wrong sign or index, or a transposed operand
can slip through would not pin the oracle; every mutant below must make at
least one pin of tests/oracle_pins.py fail.
"""
import pytest

import oracle
from oracle import modarith, ntt, polymul, roots

from .oracle_pins import ALL_PINS


def _cyclic_shifted_index(x, omega, q):           # omega^(j(k+1)) instead of omega^(jk)
    n = len(x)
    return [sum(x[j] * pow(omega, j * (k + 1), q) for j in range(n)) % q for k in range(n)]


def _cyclic_transposed(x, omega, q):              # x_k omega^(jk) summed over k, indexed by j
    n = len(x)
    return [sum(x[n - 1 - j] * pow(omega, j * k, q) for j in range(n)) % q for k in range(n)]


def _negacyclic_untwisted(a, q, psi=None):        # dropped the psi^j twist
    n = len(a)
    psi = roots.canonical_psi(q, n) if psi is None else psi
    return ntt.ntt_cyclic(list(a), psi * psi % q, q)


def _negacyclic_twist_off_by_one(a, q, psi=None):  # twist psi^(j+1)
    n = len(a)
    psi = roots.canonical_psi(q, n) if psi is None else psi
    return ntt.ntt_cyclic([a[j] * pow(psi, j + 1, q) % q for j in range(n)], psi * psi % q, q)


def _intt_no_scale(A, q, psi=None):               # forgot N^-1
    n = len(A)
    psi = roots.canonical_psi(q, n) if psi is None else psi
    pi = pow(psi, -1, q)
    y = ntt.ntt_cyclic(list(A), pi * pi % q, q)
    return [y[j] * pow(pi, j, q) % q for j in range(n)]


def _intt_wrong_untwist(A, q, psi=None):          # untwist by psi^+j
    n = len(A)
    psi = roots.canonical_psi(q, n) if psi is None else psi
    pi = pow(psi, -1, q)
    y = ntt.ntt_cyclic(list(A), pi * pi % q, q)
    return [y[j] * pow(psi, j, q) % q * pow(n, -1, q) % q for j in range(n)]


def _psi_not_minimal(q, n):                       # first root found, not the canonical one
    g = 2
    while pow(g, (q - 1) // 2, q) != q - 1:
        g += 1
    return pow(g, (q - 1) // (2 * n), q)


def _psi_cyclic_root(q, n):                       # an N-th root instead of a 2N-th root
    return pow(_psi_not_minimal(q, n), 2, q)


def _negacyclic_plus_wrap(a, b, q):               # cyclic wrap X^N = +1
    n = len(a)
    full = polymul.schoolbook(a, b, q)
    out = full[:n]
    for k in range(n, len(full)):
        out[k - n] += full[k]
    return [c % q for c in out]


def _negacyclic_at_sign(a, b, q, ks):
    n = len(a)
    return [sum(a[i] * (b[k - i] if k >= i else b[k - i + n]) for i in range(n)) % q for k in ks]


def _submod_swapped(a, b, q):
    return (b - a) % q


def _addmod_no_reduce_tie(a, b, q):               # '>' instead of '>=' in Eq. saddmod
    s = a + b
    return s - q if s > q else s


def _mulmod_dropped_term(a, b, q):                # schoolbook product missing a cross term
    lo = (1 << 64) - 1
    a0, a1, b0, b1 = a >> 64, a & lo, b >> 64, b & lo
    return ((a0 * b0 << 128) + (a0 * b1 << 64) + a1 * b1) % q


def _axpy_swapped(alpha, x, y, q):
    return [(alpha * yi + xi) % q for xi, yi in zip(x, y)]


def _forward_at_even(a, q, ks, psi=None):         # psi^(2k) instead of psi^(2k+1)
    n = len(a)
    psi = roots.canonical_psi(q, n) if psi is None else psi
    return [sum(a[j] * pow(psi, 2 * k * j, q) for j in range(n)) % q for k in ks]


MUTANTS = {
    "cyclic_shifted_index": (ntt, "ntt_cyclic", _cyclic_shifted_index),
    "cyclic_transposed": (ntt, "ntt_cyclic", _cyclic_transposed),
    "negacyclic_untwisted": (ntt, "ntt_negacyclic", _negacyclic_untwisted),
    "negacyclic_twist_off_by_one": (ntt, "ntt_negacyclic", _negacyclic_twist_off_by_one),
    "intt_no_scale": (ntt, "intt_negacyclic", _intt_no_scale),
    "intt_wrong_untwist": (ntt, "intt_negacyclic", _intt_wrong_untwist),
    "psi_not_minimal": (roots, "canonical_psi", _psi_not_minimal),
    "psi_cyclic_root": (roots, "canonical_psi", _psi_cyclic_root),
    "negacyclic_plus_wrap": (polymul, "negacyclic", _negacyclic_plus_wrap),
    "negacyclic_at_sign": (polymul, "negacyclic_at", _negacyclic_at_sign),
    "submod_swapped": (modarith, "submod", _submod_swapped),
    "addmod_tie": (modarith, "addmod", _addmod_no_reduce_tie),
    "mulmod_dropped_term": (modarith, "mulmod", _mulmod_dropped_term),
    "axpy_swapped": (modarith, "vec_axpymod", _axpy_swapped),
    "forward_at_even": (ntt, "forward_at", _forward_at_even),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, monkeypatch):
    mod, attr, fn = MUTANTS[name]
    monkeypatch.setattr(mod, attr, fn)
    caught = []
    for pin in ALL_PINS:
        try:
            pin(oracle)
        except (AssertionError, ValueError, ZeroDivisionError):
            caught.append(pin.__name__)
    assert caught, f"mutant {name} passed every pin"
