"""Element-wise modular BLAS on the GPU against the oracle, bit for bit.

Covers the three widths (60-bit moduli in one limb, 124-bit in two, 225- and
252-bit in four), odd moduli at every position of each width class (2 to 252
bits), lengths that are multiples of the kernel's chunk and ragged ones, the
paper scale length 2^16, a long ragged vector spanning 1025 blocks (sampled),
every pair of edge residues, exact aliasing (c == a) and edge scalars for
axpy."""
import itertools

import pytest

import oracle
from paper_2509_12494_amd import mwntt
from paper_2509_12494_amd import workloads as W

from .gpu_util import announce, dev, edge_values, host_ints, prime, require_gpu

pytestmark = pytest.mark.gpu

WIDTHS = [(60, 11), (124, 12), (124, 2001), (97, 13), (33, 14), (252, 15), (225, 16)]
SIZES = [1, 7, 1024, 1024 + 37, 3 * 4096 + 5, 1 << 16]
OPS = ["vec_addmod", "vec_submod", "vec_mulmod"]


def _oracle(op, a, b, q):
    return getattr(oracle.modarith, op)(a, b, q)


@pytest.mark.parametrize("bits,seed", WIDTHS)
@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("op", OPS)
def test_binary_ops(op, n, bits, seed):
    require_gpu()
    import torch
    q = prime(bits, seed)
    limbs = W.limbs_for_bits(bits)
    g = W.rng(n * 7 + bits)
    A = W.uniform_residues(g, q, n, limbs)
    B = W.uniform_residues(g, q, n, limbs)
    announce(op, n, bits)
    a, b = dev(A), dev(B)
    c = torch.empty_like(a)
    getattr(mwntt, op)(c, a, b, q, limbs)
    torch.cuda.synchronize()
    assert host_ints(c, limbs) == _oracle(op, W.to_ints(A), W.to_ints(B), q)


@pytest.mark.parametrize("bits,seed", [(60, 11), (124, 12), (252, 15)])
def test_long_vector_sampled(bits, seed):
    """n = 2^20 + 333: 1024 full blocks plus a ragged tail; every 997th
    element and the whole tail against the oracle."""
    require_gpu()
    import torch
    q = prime(bits, seed)
    limbs = W.limbs_for_bits(bits)
    n = (1 << 20) + 333
    g = W.rng(8080 + bits)
    A = W.uniform_residues(g, q, n, limbs)
    B = W.uniform_residues(g, q, n, limbs)
    alpha = W.uniform_scalar(g, q, limbs)
    a, b = dev(A), dev(B)
    ks = list(range(0, n, 997)) + list(range(n - 400, n))
    sa, sb = W.to_ints(A[ks]), W.to_ints(B[ks])

    def sampled(t):
        return W.to_ints(mwntt.to_host(t).reshape(-1, limbs)[ks])
    for op in OPS:
        announce("long", op, bits)
        c = torch.empty_like(a)
        getattr(mwntt, op)(c, a, b, q, limbs)
        torch.cuda.synchronize()
        assert sampled(c) == _oracle(op, sa, sb, q), op
    announce("long axpy", bits)
    y = b.clone()
    mwntt.vec_axpymod(y, alpha, a, q, limbs)
    torch.cuda.synchronize()
    assert sampled(y) == oracle.modarith.vec_axpymod(alpha, sa, sb, q)


@pytest.mark.parametrize("bits,seed", WIDTHS)
@pytest.mark.parametrize("n", SIZES)
def test_axpy(n, bits, seed):
    require_gpu()
    import torch
    q = prime(bits, seed)
    limbs = W.limbs_for_bits(bits)
    g = W.rng(n * 11 + bits)
    X = W.uniform_residues(g, q, n, limbs)
    Y = W.uniform_residues(g, q, n, limbs)
    alpha = W.uniform_scalar(g, q, limbs)
    announce("axpy", n, bits)
    x, y = dev(X), dev(Y)
    mwntt.vec_axpymod(y, alpha, x, q, limbs)
    torch.cuda.synchronize()
    assert host_ints(y, limbs) == oracle.modarith.vec_axpymod(alpha, W.to_ints(X), W.to_ints(Y), q)


@pytest.mark.parametrize("bits,seed", WIDTHS)
def test_edge_pairs(bits, seed):
    require_gpu()
    import torch
    q = prime(bits, seed)
    limbs = W.limbs_for_bits(bits)
    ev = edge_values(q)
    pairs = list(itertools.product(ev, ev))
    a_i = [x for x, _ in pairs]
    b_i = [y for _, y in pairs]
    a, b = dev(W.from_ints(a_i, limbs)), dev(W.from_ints(b_i, limbs))
    for op in OPS:
        announce("edge", op, bits)
        c = torch.empty_like(a)
        getattr(mwntt, op)(c, a, b, q, limbs)
        torch.cuda.synchronize()
        assert host_ints(c, limbs) == _oracle(op, a_i, b_i, q), op
    for alpha in ev:
        announce("edge axpy", alpha, bits)
        y = b.clone()
        mwntt.vec_axpymod(y, alpha, a, q, limbs)
        torch.cuda.synchronize()
        assert host_ints(y, limbs) == oracle.modarith.vec_axpymod(alpha, a_i, b_i, q)


@pytest.mark.parametrize("bits,seed", [(60, 11), (124, 12), (252, 15)])
def test_in_place_aliasing(bits, seed):
    require_gpu()
    import torch
    q = prime(bits, seed)
    limbs = W.limbs_for_bits(bits)
    n = 5000
    g = W.rng(99)
    A = W.uniform_residues(g, q, n, limbs)
    B = W.uniform_residues(g, q, n, limbs)
    for op in OPS:
        announce("alias", op, bits)
        a, b = dev(A), dev(B)
        getattr(mwntt, op)(a, a, b, q, limbs)          # c == a
        getattr(mwntt, op)(b, a, b, q, limbs)          # c == b
        torch.cuda.synchronize()
        first = _oracle(op, W.to_ints(A), W.to_ints(B), q)
        assert host_ints(a, limbs) == first
        assert host_ints(b, limbs) == _oracle(op, first, W.to_ints(B), q)


def test_sub_range_of_buffer():
    """n smaller than the buffer: residues past n are untouched."""
    require_gpu()
    import torch
    q = prime(124, 12)
    A = W.uniform_residues(W.rng(5), q, 3000, 2)
    a = dev(A)
    c = torch.zeros_like(a)
    mwntt.vec_addmod(c, a, a, q, 2, n=2049)
    torch.cuda.synchronize()
    got = host_ints(c, 2)
    assert got[:2049] == oracle.modarith.vec_addmod(W.to_ints(A)[:2049], W.to_ints(A)[:2049], q)
    assert got[2049:] == [0] * (3000 - 2049)


# Odd moduli across every width class, including the low end of each class
# and widths between the old fixed-offset Barrett ranges: 2-, 14-, 17- and
# 32-bit values written out (Barrett needs an odd modulus, not a prime), the
# rest seeded primes.
FIXED_MODULI = {2: 3, 14: 12289, 17: 65537, 32: (1 << 32) - 5}
ANY_WIDTH = [2, 14, 17, 32, 33, 59, 60, 61, 80, 96, 97, 123, 124, 125, 160, 200, 224, 225, 251, 252]


def _any_modulus(bits):
    return FIXED_MODULI.get(bits) or prime(bits, 700 + bits)


@pytest.mark.parametrize("bits", ANY_WIDTH)
def test_every_width_edges_and_ragged(bits):
    """All four ops at every width class position: every pair of edge
    residues, then a ragged uniform vector (n = 4099) and the 2^16 length,
    whole outputs against the oracle (Barrett holds for general moduli,
    Eq. barrett)."""
    require_gpu()
    import torch
    q = _any_modulus(bits)
    assert q.bit_length() == bits and q % 2 == 1
    limbs = W.limbs_for_bits(bits)
    ev = sorted(set(v % q for v in edge_values(q)))
    pairs = list(itertools.product(ev, ev))
    a_i = [x for x, _ in pairs]
    b_i = [y for _, y in pairs]
    for n, (A, B) in (("edges", (W.from_ints(a_i, limbs), W.from_ints(b_i, limbs))),
                      (4099, (W.uniform_residues(W.rng(bits), q, 4099, limbs),
                              W.uniform_residues(W.rng(bits + 1), q, 4099, limbs))),
                      (1 << 16, (W.uniform_residues(W.rng(bits + 2), q, 1 << 16, limbs),
                                 W.uniform_residues(W.rng(bits + 3), q, 1 << 16, limbs)))):
        a, b = dev(A), dev(B)
        ai, bi = W.to_ints(A), W.to_ints(B)
        for op in OPS:
            announce("any width", op, n, bits)
            c = torch.empty_like(a)
            getattr(mwntt, op)(c, a, b, q, limbs)
            torch.cuda.synchronize()
            assert host_ints(c, limbs) == _oracle(op, ai, bi, q), (op, n)
        for alpha in (ev if n == "edges" else [W.uniform_scalar(W.rng(bits + 4), q, limbs)]):
            announce("any width axpy", n, bits)
            y = b.clone()
            mwntt.vec_axpymod(y, alpha, a, q, limbs)
            torch.cuda.synchronize()
            assert host_ints(y, limbs) == oracle.modarith.vec_axpymod(alpha, ai, bi, q), (alpha, n)


@pytest.mark.parametrize("bits", [14, 33, 60, 61, 97, 124, 125, 200, 252])
def test_karatsuba_product_matches_oracle(bits):
    """vec_mulmod with the full product of its Barrett reduction formed by one
    level of Karatsuba (Eq. mulk) instead of the schoolbook columns: every
    pair of edge residues, a ragged vector and the 2^16 length, whole outputs
    against the oracle, for both products; the width's default is restored."""
    require_gpu()
    import torch
    q = _any_modulus(bits)
    limbs = W.limbs_for_bits(bits)
    ev = sorted(set(v % q for v in edge_values(q)))
    pairs = list(itertools.product(ev, ev))
    cases = [(W.from_ints([x for x, _ in pairs], limbs), W.from_ints([y for _, y in pairs], limbs))]
    for n in (4099, 1 << 16):
        cases.append((W.uniform_residues(W.rng(bits + n), q, n, limbs),
                      W.uniform_residues(W.rng(bits + n + 1), q, n, limbs)))
    default = mwntt.get_mulmod_product(limbs)
    try:
        for kara in (True, False):
            mwntt.set_mulmod_product(limbs, kara)
            assert mwntt.get_mulmod_product(limbs) is kara
            for A, B in cases:
                announce("karatsuba" if kara else "schoolbook", len(A), bits)
                a, b = dev(A), dev(B)
                c = torch.empty_like(a)
                mwntt.vec_mulmod(c, a, b, q, limbs)
                torch.cuda.synchronize()
                assert host_ints(c, limbs) == _oracle("vec_mulmod", W.to_ints(A), W.to_ints(B), q), (kara, len(A))
    finally:
        mwntt.set_mulmod_product(limbs, default)
