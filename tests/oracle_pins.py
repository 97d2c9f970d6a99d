"""Pins that tie the CPU oracle to facts fixed outside the oracle itself.

Each pin takes an oracle-like namespace (``O.modarith``, ``O.roots``, ``O.ntt``,
``O.polymul``) and raises AssertionError when the oracle disagrees with:

* the paper's worked example (Background, polynomial multiplication using NTT),
  evaluated here by direct polynomial evaluation;
* library routines on special cases (numpy integer matrix products and
  convolutions on moduli small enough for exact int64 arithmetic);
* closed forms of the transform (impulses, constants, linearity);
* brute force (order search over all of Z_q for small primes, every pair of
  residues for a small modulus, the ring definition X^N = -1);
* identities that hold at any size (INTT(NTT(a)) = a, the convolution theorem,
  Fermat's little theorem).

``tests/test_oracle.py`` runs every pin on the real oracle;
``tests/test_oracle_mutations.py`` plants plausible mistakes in copies of the
oracle and checks that at least one pin catches each of them.
"""
import json
import os
import random

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))

# Small NTT-friendly primes (q = 1 mod 2N for the listed N) for brute force.
SMALL = [(17, [1, 2, 4, 8]), (97, [1, 2, 4, 8, 16]), (193, [2, 4, 8, 16, 32]),
         (257, [4, 8, 16, 32, 64]), (7681, [2, 4, 16, 64, 256]),
         (12289, [4, 16, 64, 256])]

# Seeded primes of the workload widths (q = c*2^18 + 1), found by the seeded
# search in paper_2509_12494_amd.workloads and checked for primality there.
def wide_primes():
    from paper_2509_12494_amd import workloads as W
    return [W.find_prime(60, 7), W.find_prime(124, 8), W.find_prime(124, 2001), W.find_prime(252, 9)]


def _poly_eval(coeffs, x, q):
    """Horner evaluation, written independently of the oracle."""
    acc = 0
    for c in reversed(coeffs):
        acc = (acc * x + c) % q
    return acc


def pin_worked_example(O):
    with open(os.path.join(HERE, "golden", "worked_example_ntt.json")) as f:
        ex = json.load(f)
    q, coeffs, omega = ex["q"], ex["coefficients_low_to_high"], ex["omega"]
    # the evaluation points of the example are the powers omega^k
    pts = [pow(omega, k, q) for k in range(len(coeffs))]
    assert sorted(pts) == sorted(ex["evaluation_points"])
    want = [_poly_eval(coeffs, x, q) for x in pts]
    assert want == [2, 0, 1, 1]
    assert O.ntt.ntt_cyclic(coeffs, omega, q) == want


def pin_cyclic_vs_numpy(O):
    # Eq. (ntt) as an exact integer matrix-vector product (values < 2^31).
    for q, ns in SMALL[:5]:
        for n in ns:
            if (q - 1) % n:
                continue
            g = next(x for x in range(2, q) if all(pow(x, (q - 1) // p, q) != 1 for p in _pf(q - 1)))
            omega = pow(g, (q - 1) // n, q)
            rnd = random.Random(q * 1000 + n)
            x = [rnd.randrange(q) for _ in range(n)]
            V = np.array([[pow(omega, j * k, q) for j in range(n)] for k in range(n)], dtype=np.int64)
            want = (V @ np.array(x, dtype=np.int64)) % q
            assert O.ntt.ntt_cyclic(x, omega, q) == [int(v) for v in want]


def _pf(n):
    ps, p = [], 2
    while p * p <= n:
        while n % p == 0:
            ps.append(p)
            n //= p
        p += 1
    if n > 1:
        ps.append(n)
    return sorted(set(ps))


def pin_canonical_psi_bruteforce(O):
    for q, ns in SMALL:
        for n in ns:
            if n > 64:
                continue
            # every x in [1, q) whose order is exactly 2N: the first k with
            # x^k = 1, found by repeated multiplication (stop past 2N)
            cands = []
            for x in range(1, q):
                p, order = x, 1
                while p != 1 and order <= 2 * n:
                    p = p * x % q
                    order += 1
                if p == 1 and order == 2 * n:
                    cands.append(x)
            assert len(cands) == n
            assert O.roots.canonical_psi(q, n) == min(cands)


def pin_psi_wide(O):
    for q in wide_primes():
        for n in (2, 1 << 10, 1 << 16, 1 << 17):
            psi = O.roots.canonical_psi(q, n)
            assert 1 < psi < q
            assert pow(psi, n, q) == q - 1 and pow(psi, 2 * n, q) == 1


def pin_impulses(O):
    for q in [12289] + wide_primes():
        for n in (4, 16, 64):
            psi = O.roots.canonical_psi(q, n)
            d0 = [1] + [0] * (n - 1)
            assert O.ntt.ntt_negacyclic(d0, q) == [1] * n
            c = q - 2
            assert O.ntt.ntt_negacyclic([c] + [0] * (n - 1), q) == [c] * n
            for j in (1, 3, n - 1):
                dj = [0] * n
                dj[j] = 1
                want = [pow(psi, j * (2 * k + 1), q) for k in range(n)]
                assert O.ntt.ntt_negacyclic(dj, q) == want
            # inverse of all-ones is the unit impulse
            assert O.ntt.intt_negacyclic([1] * n, q) == d0


def pin_evaluation(O):
    # A_k = a(psi^(2k+1)): the transform evaluates the polynomial at the odd
    # powers of psi, i.e. at the N roots of X^N + 1.
    for q in [7681] + wide_primes():
        for n in (8, 32, 128):
            rnd = random.Random(n + q % 1000)
            a = [rnd.randrange(q) for _ in range(n)]
            psi = O.roots.canonical_psi(q, n)
            want = [_poly_eval(a, pow(psi, 2 * k + 1, q), q) for k in range(n)]
            for k in range(n):
                r = pow(psi, 2 * k + 1, q)
                assert pow(r, n, q) == q - 1          # r is a root of X^N + 1
            assert O.ntt.ntt_negacyclic(a, q) == want
            ks = [0, 1, n // 2, n - 1]
            assert O.ntt.forward_at(a, q, ks) == [want[k] for k in ks]


def pin_roundtrip_linearity(O):
    for q in wide_primes():
        for n in (2, 16, 256):
            rnd = random.Random(q % 997 + n)
            a = [rnd.randrange(q) for _ in range(n)]
            b = [rnd.randrange(q) for _ in range(n)]
            A = O.ntt.ntt_negacyclic(a, q)
            assert O.ntt.intt_negacyclic(A, q) == a
            B = O.ntt.ntt_negacyclic(b, q)
            s = [(x + y) % q for x, y in zip(a, b)]
            assert O.ntt.ntt_negacyclic(s, q) == [(x + y) % q for x, y in zip(A, B)]
            js = [0, 1, n - 1]
            assert O.ntt.inverse_at(A, q, js) == [a[j] for j in js]


def pin_negacyclic_product_ring(O):
    # X^(N-1) * X = X^N = -1 in Z_q[X]/(X^N + 1)
    for q in [17] + wide_primes()[:1]:
        n = 8
        a = [0] * (n - 1) + [1]
        b = [0, 1] + [0] * (n - 2)
        assert O.polymul.negacyclic(a, b, q) == [q - 1] + [0] * (n - 1)
    # numpy convolution, then fold with X^N = -1 (exact int64, small q)
    for q, n in ((17, 8), (257, 64), (7681, 32)):
        rnd = random.Random(q + n)
        a = [rnd.randrange(q) for _ in range(n)]
        b = [rnd.randrange(q) for _ in range(n)]
        full = np.convolve(np.array(a, dtype=np.int64), np.array(b, dtype=np.int64))
        want = full[:n].copy()
        want[: n - 1] -= full[n:]
        want %= q
        assert O.polymul.negacyclic(a, b, q) == [int(v) for v in want]
        ks = [0, 5, n - 1]
        assert O.polymul.negacyclic_at(a, b, q, ks) == [int(want[k]) for k in ks]


def pin_convolution_theorem(O):
    for q in [12289] + wide_primes():
        for n in (4, 32, 128):
            rnd = random.Random(7 * n + q % 101)
            a = [rnd.randrange(q) for _ in range(n)]
            b = [rnd.randrange(q) for _ in range(n)]
            A, B = O.ntt.ntt_negacyclic(a, q), O.ntt.ntt_negacyclic(b, q)
            c = O.ntt.intt_negacyclic([x * y % q for x, y in zip(A, B)], q)
            assert c == O.polymul.negacyclic(a, b, q)


def pin_blas_bruteforce_small(O):
    q = 17
    M = O.modarith
    for a in range(q):
        for b in range(q):
            s, d, p = M.addmod(a, b, q), M.submod(a, b, q), M.mulmod(a, b, q)
            assert 0 <= s < q and (s - a - b) % q == 0
            assert 0 <= d < q and (d + b - a) % q == 0 and M.addmod(d, b, q) == a
            assert 0 <= p < q and (p - a * b) % q == 0


def pin_blas_special(O):
    M = O.modarith
    for q in wide_primes():
        rnd = random.Random(q % 12345)
        a = [rnd.randrange(q) for _ in range(64)] + [0, 1, q - 1, q - 2]
        n = len(a)
        neg = [(q - x) % q for x in a]
        assert M.vec_addmod(a, neg, q) == [0] * n          # a + (q - a) = 0 (tie -> 0)
        assert M.vec_submod(a, a, q) == [0] * n
        assert M.vec_submod([0] * n, a, q) == neg
        assert M.vec_mulmod(a, [1] * n, q) == a
        assert M.vec_mulmod(a, [0] * n, q) == [0] * n
        assert M.mulmod(q - 1, q - 1, q) == 1                # (-1)^2 = 1
        inv = [pow(x, -1, q) if x else 0 for x in a]
        assert M.vec_mulmod(a, inv, q) == [1 if x else 0 for x in a]
        # Fermat: a^(q-1) = 1 by square-and-multiply on the oracle's mulmod
        for x in a[:4]:
            if x == 0:
                continue
            r, base, e = 1, x, q - 1
            while e:
                if e & 1:
                    r = M.mulmod(r, base, q)
                base = M.mulmod(base, base, q)
                e >>= 1
            assert r == 1
        y = a[::-1]
        assert M.vec_axpymod(0, a, y, q) == y
        assert M.vec_axpymod(1, a, y, q) == M.vec_addmod(a, y, q)
        assert M.vec_axpymod(q - 1, a, a, q) == [0] * n      # -x + x = 0
        alpha = rnd.randrange(q)
        assert M.vec_axpymod(alpha, [0] * n, y, q) == y
        two = M.vec_axpymod(alpha, a, [0] * n, q)
        assert two == M.vec_mulmod([alpha] * n, a, q)


ALL_PINS = [pin_worked_example, pin_cyclic_vs_numpy, pin_canonical_psi_bruteforce,
            pin_psi_wide, pin_impulses, pin_evaluation, pin_roundtrip_linearity,
            pin_negacyclic_product_ring, pin_convolution_theorem,
            pin_blas_bruteforce_small, pin_blas_special]
