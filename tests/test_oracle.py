"""The CPU oracle against its pins (no GPU)."""
import pytest

import oracle
from paper_2509_12494_amd import workloads as W
from sympy import isprime

from .oracle_pins import ALL_PINS


@pytest.mark.parametrize("pin", ALL_PINS, ids=lambda p: p.__name__)
def test_pin(pin):
    pin(oracle)


@pytest.mark.parametrize("bits,seed", [(60, 1), (60, 3001), (124, 1001), (124, 2001), (124, 4001)])
def test_seeded_prime(bits, seed):
    q = W.find_prime(bits, seed)
    assert isprime(q) and q.bit_length() == bits and q % (1 << 18) == 1
    assert q == W.find_prime(bits, seed)          # deterministic


def test_uniform_residues_canonical_and_seeded():
    q = W.find_prime(124, 11)
    a = W.uniform_residues(W.rng(5), q, 5000, 2)
    b = W.uniform_residues(W.rng(5), q, 5000, 2)
    assert (a == b).all()
    vals = W.to_ints(a)
    assert all(0 <= v < q for v in vals)
    # top bits are exercised (values above q/2 occur) and round-trip exactly
    assert max(vals) > q // 2 and min(vals) < q // 2
    assert (W.from_ints(vals, 2) == a).all()


def test_direct_and_indexed_forms_agree():
    q = W.find_prime(124, 2001)
    n = 1 << 9
    a = W.to_ints(W.uniform_residues(W.rng(9), q, n, 2))
    A = oracle.ntt.ntt_negacyclic(a, q)
    ks = [0, 1, 17, 255, 511]
    assert oracle.ntt.forward_at(a, q, ks) == [A[k] for k in ks]
    assert oracle.ntt.inverse_at(A, q, ks) == [a[k] for k in ks]


def test_oracle_rejects_bad_inputs():
    q = W.find_prime(60, 1)
    with pytest.raises(ValueError):
        oracle.ntt.ntt_negacyclic([q] + [0] * 7, q)
    with pytest.raises(ValueError):
        oracle.ntt.ntt_negacyclic([0] * 6, q)
    v = ((q - 1) & -(q - 1)).bit_length() - 1       # 2-adic valuation of q - 1
    with pytest.raises(ValueError):
        oracle.roots.canonical_psi(q, 1 << v)         # needs 2N | q - 1
