"""Roots of unity for the length-N negacyclic transform.

Eq. (ntt) uses "the n-th primitive root of unity" without saying which one.
For the negacyclic transform of length N the oracle needs a primitive 2N-th
root psi (psi^N = -1), with omega_N = psi^2 playing the role of Eq. (ntt)'s
root.  Any of the N primitive 2N-th roots gives a correct but different
transform, so the oracle fixes one reading, the *canonical* root: the smallest
integer in [1, q) whose multiplicative order is exactly 2N.

Construction (all by definition):
* the modulus must satisfy q = 1 (mod 2N) for such a root to exist;
* g = smallest integer >= 2 with g^((q-1)/2) = -1 (a quadratic non-residue);
  then psi0 = g^((q-1)/(2N)) satisfies psi0^N = g^((q-1)/2) = -1, so its order
  is exactly 2N (2N is a power of two, and psi0^N != 1);
* the primitive 2N-th roots are exactly psi0^(2i+1), 0 <= i < N; the canonical
  root is the minimum of that set (independent of g).

Parity pins: tests/test_oracle.py (brute-force order search over all of Z_q
for small primes; psi^N = -1 and psi^2N = 1 at the workload widths).
"""


def check_ntt_modulus(q: int, n: int) -> None:
    if n < 1 or n & (n - 1):
        raise ValueError("N must be a power of two")
    if q < 3 or q % 2 == 0:
        raise ValueError("modulus must be an odd integer >= 3")
    if (q - 1) % (2 * n):
        raise ValueError("modulus must satisfy q = 1 mod 2N")


def canonical_psi(q: int, n: int) -> int:
    """Smallest primitive 2N-th root of unity modulo the prime q."""
    check_ntt_modulus(q, n)
    g = 2
    while pow(g, (q - 1) // 2, q) != q - 1:
        g += 1
    psi0 = pow(g, (q - 1) // (2 * n), q)
    if pow(psi0, n, q) != q - 1:
        raise ValueError("no primitive 2N-th root found (is q prime?)")
    best = psi0
    sq = psi0 * psi0 % q
    cur = psi0
    for _ in range(1, n):
        cur = cur * sq % q          # psi0^(2i+1)
        if cur < best:
            best = cur
    return best

