"""The scalar C++ CPU baseline (cpu_ref) against the oracle, on the CPU: its
canonical root is the oracle's; whole forward and inverse transforms equal
the oracle's at N = 2^1 .. 2^9 for one-, two- and four-word moduli (at the
top of each class and inside it); a 2^16 124-bit transform matches the oracle
on sampled outputs and round-trips; the BLAS operations equal the oracle on
edge and random operands; threaded calls equal single-threaded ones; invalid
arguments are refused.  Also: neither the GPU package nor the oracle imports
the baseline or each other's code."""
import os
import re

import numpy as np
import pytest

import cpu_ref
import oracle
from paper_2509_12494_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module", autouse=True)
def built():
    if not os.path.exists(cpu_ref.LIB):
        cpu_ref.build()


def _arr(xs, limbs):
    return W.from_ints(list(xs), limbs)


def _ints(a):
    return W.to_ints(a)


WIDTHS = [(33, 1), (60, 1), (80, 2), (124, 2), (200, 4), (252, 4)]


@pytest.mark.parametrize("bits,limbs", WIDTHS)
def test_root_and_small_transforms_equal_oracle(bits, limbs):
    q = W.find_prime(bits, 300 + bits)
    g = W.rng(bits)
    for log2n in range(1, 10):
        n = 1 << log2n
        p = cpu_ref.Plan(log2n, q, limbs)
        assert p.root() == oracle.roots.canonical_psi(q, n)
        a = W.uniform_residues(g, q, n, limbs)
        A = p.transform(a)
        assert _ints(A) == oracle.ntt.ntt_negacyclic(_ints(a), q), (bits, log2n)
        back = p.transform(A, inverse=True)
        assert _ints(back) == _ints(a)
        assert _ints(p.transform(a, inverse=True)) == oracle.ntt.intt_negacyclic(_ints(a), q), (bits, log2n)
        p.destroy()


def test_given_root_is_used():
    q = W.find_prime(124, 7)
    n = 1 << 6
    psi = pow(oracle.roots.canonical_psi(q, n), 5, q)   # another primitive 2N-th root
    p = cpu_ref.Plan(6, q, 2, psi=psi)
    a = W.uniform_residues(W.rng(8), q, n, 2)
    assert _ints(p.transform(a)) == oracle.ntt.ntt_negacyclic(_ints(a), q, psi=psi)


def test_paper_size_sampled_and_round_trip():
    q = W.find_prime(124, 2001)
    n = 1 << 16
    a = W.uniform_residues(W.rng(2001), q, n, 2)
    p = cpu_ref.Plan(16, q, 2)
    A = p.transform(a)
    ks = [0, 1, 2, 777, n // 2, n - 2, n - 1, 40961]
    got = _ints(A)
    assert [got[k] for k in ks] == oracle.ntt.forward_at(_ints(a), q, ks)
    assert np.array_equal(p.transform(A, inverse=True), a)


@pytest.mark.parametrize("bits,limbs", WIDTHS)
def test_blas_equals_oracle(bits, limbs):
    q = W.find_prime(bits, 400 + bits)
    g = W.rng(bits + 1)
    edges = [0, 1, 2, q - 1, q - 2, (q - 1) // 2, (q + 1) // 2]
    xa = [x for x in edges for _ in edges] + _ints(W.uniform_residues(g, q, 1000, limbs))
    xb = [y for _ in edges for y in edges] + _ints(W.uniform_residues(g, q, 1000, limbs))
    a, b = _arr(xa, limbs), _arr(xb, limbs)
    alpha = W.uniform_scalar(g, q, limbs)
    assert _ints(cpu_ref.blas("add", a, b, q, limbs)) == oracle.modarith.vec_addmod(xa, xb, q)
    assert _ints(cpu_ref.blas("sub", a, b, q, limbs)) == oracle.modarith.vec_submod(xa, xb, q)
    assert _ints(cpu_ref.blas("mul", a, b, q, limbs)) == oracle.modarith.vec_mulmod(xa, xb, q)
    assert _ints(cpu_ref.blas("axpy", a, b, q, limbs, alpha=alpha)) == oracle.modarith.vec_axpymod(alpha, xa, xb, q)
    for al in (0, 1, q - 1):
        assert _ints(cpu_ref.blas("axpy", a, b, q, limbs, alpha=al)) == oracle.modarith.vec_axpymod(al, xa, xb, q)


def test_threads_match_single_thread():
    q = W.find_prime(124, 11)
    g = W.rng(12)
    p = cpu_ref.Plan(10, q, 2)
    a = W.uniform_residues(g, q, 7 << 10, 2)
    assert np.array_equal(p.transform(a, threads=4), p.transform(a, threads=1))
    assert np.array_equal(p.transform(a, inverse=True, threads=0), p.transform(a, inverse=True, threads=1))
    x, y = W.uniform_residues(g, q, 50001, 2), W.uniform_residues(g, q, 50001, 2)
    assert np.array_equal(cpu_ref.blas("mul", x, y, q, 2, threads=5), cpu_ref.blas("mul", x, y, q, 2, threads=1))


def test_invalid_arguments():
    q = W.find_prime(124, 13)
    with pytest.raises(RuntimeError):
        cpu_ref.Plan(6, q + 1, 2)                 # even
    with pytest.raises(RuntimeError):
        cpu_ref.Plan(6, q, 1)                     # 124 bits in one word
    with pytest.raises(RuntimeError):
        cpu_ref.Plan(6, q, 2, psi=1)              # not a primitive 2N-th root
    with pytest.raises(RuntimeError):
        cpu_ref.Plan(18, q, 2)                    # N > 2^17
    x = W.uniform_residues(W.rng(1), q, 8, 2)
    with pytest.raises(RuntimeError):
        cpu_ref.blas("axpy", x, x, q, 2, alpha=q)  # alpha not reduced


def _imports(path):
    src = open(path).read()
    return set(re.findall(r"^\s*(?:from|import)\s+([A-Za-z_][\w.]*)", src, re.M))


def test_code_separation():
    """The GPU package never imports the oracle or the CPU baseline, and the
    oracle imports neither of them."""
    pkg = os.path.join(ROOT, "paper_2509_12494_amd")
    for f in os.listdir(pkg):
        if f.endswith(".py"):
            mods = _imports(os.path.join(pkg, f))
            assert not any(m.split(".")[0] in ("oracle", "cpu_ref") for m in mods), f
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith(".py"):
            mods = _imports(os.path.join(ROOT, "oracle", f))
            assert not any(m.split(".")[0] in ("paper_2509_12494_amd", "cpu_ref") for m in mods), f
