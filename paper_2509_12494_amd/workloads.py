"""Seeded synthetic inputs shared by the tests, the oracle checks and the benchmark.

This module only draws numbers: NTT-friendly primes found by a seeded search,
residues drawn uniformly from [0, q) by rejection, and the mixed batch and
request-stream recipes.  It holds none of the transform or modular arithmetic
of the method; the HIP path and the CPU oracle each implement that on their own
and both consume the values drawn here.

Representation.  A residue of a modulus with ``limbs`` 64-bit words is stored
as ``limbs`` little-endian ``uint64`` words (word 0 = least significant), so a
length-n vector is a ``numpy.uint64`` array of shape ``(n, limbs)``.  The paper
writes a double-word as ``[x0, x1]`` with ``x0`` the HIGH word (Background,
double-word arithmetic, Eq. def_dw); that is notation only, memory here is
little-endian.

Prime recipe: q = c * 2^m + 1 with c drawn uniformly from
[2^(b-1-m), 2^(b-m)) by a PCG64 stream, redrawn until q is prime (sympy's
BPSW test).  That gives bitlen(q) = b and q = 1 (mod 2^m); m = 18 makes every
N <= 2^17 NTT-friendly (q = 1 mod 2N).  b = 124 is the largest width Barrett
reduction allows for 128-bit arithmetic (Background, modular arithmetic); b = 60
is the same rule applied to one 64-bit word and b = 252 to four words (the
larger widths the paper names as a next step, Discussion).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence

import numpy as np
from sympy import isprime

__all__ = [
    "rng", "limbs_for_bits", "find_prime", "uniform_residues", "uniform_ints", "to_ints",
    "from_ints", "uniform_scalar", "Workload", "config_small", "config_paper",
    "config_batched", "config_fused", "config_rns", "serving_stream", "PRIME_M",
]

PRIME_M = 18  # q = 1 mod 2^18 for every seeded prime


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def limbs_for_bits(bits: int) -> int:
    if bits <= 60:
        return 1
    if bits <= 124:
        return 2
    if bits <= 252:
        return 4
    raise ValueError("moduli above 252 bits are not supported")


def _draw_bits(g: np.random.Generator, nbits: int) -> int:
    """Uniform integer in [0, 2^nbits) from whole 64-bit draws."""
    words = (nbits + 63) // 64
    v = 0
    for w in g.integers(0, 2**64, size=words, dtype=np.uint64, endpoint=False):
        v = (v << 64) | int(w)
    return v & ((1 << nbits) - 1)


def find_prime(bits: int, seed: int, m: int = PRIME_M) -> int:
    """Seeded search for a prime q = c*2^m + 1 with bitlen(q) == bits."""
    if bits - 1 - m < 1:
        raise ValueError("bits too small for the requested 2-power factor")
    g = rng(seed)
    lo = 1 << (bits - 1 - m)
    while True:
        c = lo + _draw_bits(g, bits - 1 - m)
        q = (c << m) | 1
        if isprime(q):
            return q


def uniform_residues(g: np.random.Generator, q: int, n: int, limbs: int) -> np.ndarray:
    """n residues uniform in [0, q) as a (n, limbs) uint64 array (rejection sampling).

    Each candidate draws the nw = ceil(bitlen(q) / 64) significant words, masks
    the top one to the bit length of q minus 64*(nw-1) bits and is redrawn when
    >= q (acceptance >= 1/2); words above nw are zero.
    """
    bl = q.bit_length()
    nw = (bl + 63) // 64
    if not 1 <= nw <= limbs:
        raise ValueError("modulus width does not match the limb count")
    top_bits = bl - 64 * (nw - 1)
    top_mask = np.uint64((1 << top_bits) - 1) if top_bits < 64 else np.uint64(2**64 - 1)
    qw = [np.uint64((q >> (64 * i)) & (2**64 - 1)) for i in range(nw)]
    out = np.zeros((n, limbs), dtype=np.uint64)
    todo = np.arange(n)
    while todo.size:
        cand = g.integers(0, 2**64, size=(todo.size, nw), dtype=np.uint64, endpoint=False)
        cand[:, nw - 1] &= top_mask
        # lexicographic compare from the most significant word: cand < q
        less = np.zeros(todo.size, dtype=bool)
        equal = np.ones(todo.size, dtype=bool)
        for i in range(nw - 1, -1, -1):
            less |= equal & (cand[:, i] < qw[i])
            equal &= cand[:, i] == qw[i]
        out[todo[less], :nw] = cand[less]
        todo = todo[~less]
    return out


def uniform_ints(g: np.random.Generator, q: int, n: int) -> List[int]:
    """n Python ints uniform in [0, q) for a modulus of any width (rejection on
    ceil(bitlen(q)/64) drawn words)."""
    nw = (q.bit_length() + 63) // 64
    return to_ints(uniform_residues(g, q, n, nw))


def uniform_scalar(g: np.random.Generator, q: int, limbs: int) -> int:
    return to_ints(uniform_residues(g, q, 1, limbs))[0]


def to_ints(arr: np.ndarray) -> List[int]:
    """(n, limbs) uint64 array -> list of Python ints."""
    a = np.asarray(arr, dtype=np.uint64)
    if a.ndim == 1:
        a = a[:, None]
    res = [int(x) for x in a[:, 0]]
    for i in range(1, a.shape[1]):
        col = a[:, i]
        res = [r | (int(c) << (64 * i)) for r, c in zip(res, col)]
    return res


def from_ints(vals: Sequence[int], limbs: int) -> np.ndarray:
    """List of non-negative ints below 2^(64*limbs) -> (n, limbs) uint64 array."""
    out = np.empty((len(vals), limbs), dtype=np.uint64)
    mask = 2**64 - 1
    for i in range(limbs):
        out[:, i] = np.fromiter(((v >> (64 * i)) & mask for v in vals),
                                dtype=np.uint64, count=len(vals))
    return out


# ---------------------------------------------------------------------------
# Workload recipes.  Seeds follow config_id*1000 + index.
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Workload:
    name: str
    log2n: int
    q: int
    limbs: int
    data: dict


def config_small(seed_base: int = 1000) -> Workload:
    """One forward+inverse NTT at N=2^10 with a 124-bit prime; BLAS on length 2^10."""
    return _plain("small: N=2^10, 124-bit q", 10, 124, seed_base)


def config_paper(bits: int = 124, seed_base: int = 2000) -> Workload:
    """Forward+inverse NTT at N=2^16 with a 124-bit prime; BLAS on length 2^16."""
    return _plain(f"paper scale: N=2^16, {bits}-bit q", 16, bits, seed_base)


def _plain(name: str, log2n: int, bits: int, seed_base: int) -> Workload:
    q = find_prime(bits, seed_base + 1)
    limbs = limbs_for_bits(bits)
    g = rng(seed_base + 2)
    n = 1 << log2n
    data = {
        "poly": uniform_residues(g, q, n, limbs),
        "a": uniform_residues(g, q, n, limbs),
        "b": uniform_residues(g, q, n, limbs),
        "alpha": uniform_scalar(g, q, limbs),
    }
    return Workload(name, log2n, q, limbs, data)


def config_batched(count: int = 96, seed_base: int = 3000,
                   log2n_choices: Sequence[int] = (12, 13, 14, 15, 16)):
    """Mixed batch: N_i uniform over log2n_choices, even i -> 60-bit prime, odd i -> 124-bit.

    Returns a list of (log2n, q, limbs, coeffs) tuples.
    """
    g = rng(seed_base)
    sizes = g.choice(np.asarray(log2n_choices), size=count)
    polys = []
    for i in range(count):
        bits = 60 if i % 2 == 0 else 124
        q = find_prime(bits, seed_base + 1 + i)
        limbs = limbs_for_bits(bits)
        coeffs = uniform_residues(rng(seed_base + 500 + i), q, 1 << int(sizes[i]), limbs)
        polys.append((int(sizes[i]), q, limbs, coeffs))
    return polys


def config_fused(pairs: int = 256, log2n: int = 14, seed_base: int = 4000):
    """Batched polynomial products: `pairs` pairs of N-coefficient polynomials, one 124-bit q."""
    q = find_prime(124, seed_base + 1)
    g = rng(seed_base + 2)
    n = 1 << log2n
    a = uniform_residues(g, q, pairs * n, 2).reshape(pairs, n, 2)
    b = uniform_residues(g, q, pairs * n, 2).reshape(pairs, n, 2)
    return q, a, b


def config_rns(count: int = 8, log2n: int = 16, bits: int = 124, seed_base: int = 7000):
    """RNS form of polynomials (the FHE shape): `count` NTT-friendly primes of
    `bits` bits sharing N = 2^log2n.  Returns the list of primes; a polynomial
    mod Q = prod(q_i) is held as one residue polynomial per prime."""
    return [find_prime(bits, seed_base + 1 + i) for i in range(count)]


def serving_stream(num: int, rate: float = 20000.0, seed: int = 5000,
                   min_log2: int = 10, max_log2: int = 17, primes_per_width: int = 4):
    """Poisson request stream of mixed NTT/BLAS jobs (recipe only, no inputs).

    70% NTT (half forward, half inverse) with N = 2^e, e uniform in
    [min_log2, max_log2]; 30% BLAS (half mulmod, half axpymod) with length
    floor(2^u), u uniform in [min_log2, max_log2]; width 60 or 124 bits with
    equal probability, from a pool of seeded primes per width.
    """
    g = rng(seed)
    pool = {60: [find_prime(60, seed + 100 + i) for i in range(primes_per_width)],
            124: [find_prime(124, seed + 200 + i) for i in range(primes_per_width)]}
    gaps = g.exponential(1.0 / rate, size=num)
    arrivals = np.cumsum(gaps) - gaps[0]
    jobs = []
    for i in range(num):
        is_ntt = g.random() < 0.7
        bits = 60 if g.random() < 0.5 else 124
        q = pool[bits][int(g.integers(0, primes_per_width))]
        if is_ntt:
            op = "ntt_forward" if g.random() < 0.5 else "ntt_inverse"
            size = 1 << int(g.integers(min_log2, max_log2 + 1))
        else:
            op = "vec_mulmod" if g.random() < 0.5 else "vec_axpymod"
            size = int(math.floor(2.0 ** g.uniform(min_log2, max_log2)))
        jobs.append({"t": float(arrivals[i]), "op": op, "size": size, "q": q,
                     "limbs": limbs_for_bits(bits), "seed": seed * 1000 + i})
    return jobs
