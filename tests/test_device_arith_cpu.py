"""CPU pin of the device arithmetic: mw_arith.h and mw_butterfly.h compiled for
the host (tests/host_arith/emulate.cpp, the three CDNA instruction wrappers
emulated exactly) against Python integers, at every width, at the low end,
middle and top of each width class, on edge and random operands.

What is pinned (Background, modular arithmetic: Eq. saddmod, Eq. ssubmod,
Eq. barrett; Eq. muls for the word products):
* Shoup x*w mod q up to a multiple of q, in [0, 6q) for one and two words and
  [0, 3q) for four words, for every x < 2^(32W);
* Barrett a*b mod q canonical for a, b < q (the scaled modulus below the top of
  a class), with the schoolbook and with the Karatsuba product (Eq. mulk);
* the Karatsuba full product exact for any operands below 2^(32W);
* canonical modular add and sub;
* the butterflies' congruences and lazy ranges: forward inputs [0, 16q) ->
  X' in [0, 14q), Y' in (2q, 16q); inverse inputs [0, 8q) -> X' in [0, 8q),
  Y' in [0, 6q); the last inverse stage canonical with N^-1 folded in;
* the final canonicalization from [0, 16q).
The constants (Barrett mu, the scaled modulus) come from the library's own
host code (mw_common.h), the Shoup companions from Python."""
import os
import random
import shutil
import subprocess

import pytest

from paper_2509_12494_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "host_arith")
CLANG = "/opt/rocm/llvm/bin/clang++"

# (words per residue, modulus bit widths): low end, middle and top of each
# class, with written-out small odd moduli for the one-word class
MODULI = {
    2: [3, 12289, 65537, (1 << 32) - 5, 33, 47, 59, 60],
    4: [61, 64, 80, 96, 97, 110, 123, 124],
    8: [125, 128, 160, 192, 224, 225, 251, 252],
}


def _modulus(bits_or_q):
    if bits_or_q in (3, 12289, 65537, (1 << 32) - 5):
        return bits_or_q
    return W.find_prime(bits_or_q, 1300 + bits_or_q)


@pytest.fixture(scope="module")
def emulator(tmp_path_factory):
    if not os.path.exists(CLANG) and not shutil.which("clang++"):
        pytest.fail("no clang++ for the host build of the device arithmetic")
    cxx = CLANG if os.path.exists(CLANG) else shutil.which("clang++")
    exe = str(tmp_path_factory.mktemp("emul") / "emulate")
    subprocess.run([cxx, "-O2", "-std=c++17", "-Wall", "-Werror", "-I" + os.path.join(HERE, "stub"),
                    "-I" + os.path.join(ROOT, "paper_2509_12494_amd", "csrc"), "-I" + os.path.join(ROOT, "include"),
                    os.path.join(HERE, "emulate.cpp"), "-o", exe], check=True)
    return exe


def _run(exe, lines):
    r = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True, check=True)
    out = r.stdout.splitlines()
    assert len(out) == len(lines)
    assert "error" not in out
    return [[int(x, 16) for x in o.split()] for o in out]


def _h(x):
    return format(x, "x")


def _edges(q, top):
    vals = {0, 1, 2, q - 1, q, q + 1, 2 * q - 1, 4 * q - 1, 6 * q - 1, 8 * q - 1, 8 * q, 14 * q - 1,
            16 * q - 1, top - 1, q // 2, (1 << 32) - 1, (1 << 64) - 1}
    return sorted(v for v in vals if 0 <= v < top)


@pytest.mark.parametrize("words", [2, 4, 8])
def test_device_arithmetic_on_host(emulator, words):
    rnd = random.Random(4242 + words)
    top = 1 << (32 * words)
    for spec in MODULI[words]:
        q = _modulus(spec)
        assert q % 2 == 1 and (q.bit_length() <= 32 * words - 4)
        lines, checks = [], []
        res = [v for v in _edges(q, q)] + [rnd.randrange(q) for _ in range(40)]
        lazy16 = [v for v in _edges(q, 16 * q)] + [rnd.randrange(16 * q) for _ in range(40)]
        lazy8 = [v for v in _edges(q, 8 * q)] + [rnd.randrange(8 * q) for _ in range(40)]
        anyx = [v for v in _edges(q, top)] + [rnd.randrange(top) for _ in range(40)]
        ws = [0, 1, q - 1] + [rnd.randrange(q) for _ in range(6)]

        def add(line, check):
            lines.append(f"{line[0]} {words} {_h(q)} " + " ".join(_h(v) for v in line[1:]))
            checks.append(check)

        shoup_bound = 3 * q if words == 8 else 6 * q
        for w in ws:
            wsh = (w << (32 * words)) // q
            for x in anyx[::3] + [top - 1]:
                add(("shoup", x, w, wsh),
                    lambda r, x=x, w=w: r[0] < shoup_bound and r[0] % q == x * w % q)
        for a in res[::2]:
            for b in res[1::3]:
                add(("barrett", a, b), lambda r, a=a, b=b: r[0] == a * b % q)
                add(("barrettk", a, b), lambda r, a=a, b=b: r[0] == a * b % q)
                add(("addmod", a, b), lambda r, a=a, b=b: r[0] == (a + b) % q)
                add(("submod", a, b), lambda r, a=a, b=b: r[0] == (a - b) % q)
        for w in ws[:5]:
            wsh = (w << (32 * words)) // q
            for X, Y in zip(lazy16, reversed(lazy16)):
                add(("ct", X, Y, w, wsh),
                    lambda r, X=X, Y=Y, w=w: r[0] < 14 * q and 2 * q < r[1] < 16 * q
                    and r[0] % q == (X + w * Y) % q and r[1] % q == (X - w * Y) % q)
            for X, Y in zip(lazy8, reversed(lazy8)):
                add(("gs", X, Y, w, wsh),
                    lambda r, X=X, Y=Y, w=w: r[0] < 8 * q and r[1] < 6 * q
                    and r[0] % q == (X + Y) % q and r[1] % q == (X - Y) * w % q)
        ninv = pow(1 << 10, -1, q) if q > 2 else 1
        m = ws[3] * ninv % q
        for X, Y in zip(lazy8, reversed(lazy8)):
            add(("gslast", X, Y, ninv, (ninv << (32 * words)) // q, m, (m << (32 * words)) // q),
                lambda r, X=X, Y=Y: r[0] == (X + Y) * ninv % q and r[1] == (X - Y) * m % q)
        for x in lazy16:
            add(("canon", x), lambda r, x=x: r[0] == x % q)
        for a, b in zip(anyx, reversed(anyx)):
            add(("kara", a, b), lambda r, a=a, b=b: r[0] == a * b)
        got = _run(emulator, lines)
        bad = [(ln, g) for ln, g, c in zip(lines, got, checks) if not c(g)]
        assert not bad, f"{len(bad)} of {len(lines)} cases fail at {q.bit_length()} bits, first: {bad[0]}"


def test_emulation_detects_a_planted_error(emulator, tmp_path):
    """The harness is able to fail: a copy of the header with one carry
    dropped from the Shoup quotient estimate gives wrong results."""
    src = os.path.join(ROOT, "paper_2509_12494_amd", "csrc")
    work = tmp_path / "pkg" / "csrc"                   # keeps csrc/../../include resolvable
    shutil.copytree(src, work)
    shutil.copytree(os.path.join(ROOT, "include"), tmp_path / "include")
    text = (work / "mw_arith.h").read_text()
    needle = "  // column 4\n  acc = pack(hi32(acc), t);"
    assert needle in text
    (work / "mw_arith.h").write_text(text.replace(needle, "  // column 4\n  acc = pack(hi32(acc), 0u);"))
    exe = str(tmp_path / "emulate_bad")
    cxx = CLANG if os.path.exists(CLANG) else shutil.which("clang++")
    subprocess.run([cxx, "-O2", "-std=c++17", "-I" + os.path.join(HERE, "stub"), "-I" + str(work),
                    "-I" + os.path.join(ROOT, "include"), os.path.join(HERE, "emulate.cpp"), "-o", exe], check=True)
    q = W.find_prime(124, 1424)
    rnd = random.Random(1)
    lines, want = [], []
    for _ in range(200):
        x, w = rnd.randrange(1 << 128), rnd.randrange(q)
        lines.append(f"shoup 4 {_h(q)} {_h(x)} {_h(w)} {_h((w << 128) // q)}")
        want.append((x * w) % q)
    got = _run(exe, lines)
    assert any(g[0] % q != v or g[0] >= 6 * q for g, v in zip(got, want))


@pytest.mark.parametrize("words", [2, 4, 8])
def test_canonicalisation_around_every_multiple(emulator, words):
    """canon16 from [0, 16q) to [0, q): x = kq - 1, kq, kq + 1 for every k in
    1..15, the ends of the range and random values, for moduli whose top word
    is just below and at 2^16 (the quotient estimate's threshold), well inside
    and at the top of the width class (bit length 32 W - 4)."""
    rnd = random.Random(77 + words)
    base = 32 * (words - 1)
    moduli = [
        (((1 << 16) - 1) << base) | 1 | (rnd.getrandbits(base) | 1),   # top word 2^16 - 1: four subtractions
        ((1 << 16) << base) | 1,                                        # top word 2^16: the estimate, smallest
        ((1 << 16) << base) | (rnd.getrandbits(base) | 1),
        (rnd.randrange(1 << 20, 1 << 27) << base) | (rnd.getrandbits(base) | 1),
        (1 << (32 * words - 4)) - 1,                                    # largest odd modulus of the class
        ((1 << 27) << base) | 1,                                        # smallest with a full top word
    ]
    for q in moduli:
        assert q % 2 == 1 and q.bit_length() <= 32 * words - 4
        xs = {0, 1, q - 1, 16 * q - 1, 16 * q - 2}
        for k in range(1, 16):
            xs |= {k * q - 1, k * q, k * q + 1}
        xs = sorted(x for x in xs if 0 <= x < 16 * q) + [rnd.randrange(16 * q) for _ in range(300)]
        lines = [f"canon {words} {_h(q)} {_h(x)}" for x in xs]
        got = _run(emulator, lines)
        bad = [(hex(x), g) for x, g in zip(xs, got) if g[0] != x % q]
        assert not bad, f"{len(bad)} of {len(xs)} wrong for q = {hex(q)}, first: {bad[0]}"


def test_canonicalisation_detects_a_planted_error(tmp_path):
    """The canonicalisation pin is able to fail: a copy whose quotient-estimate
    reciprocal is rounded up instead of down gives wrong results just below
    the multiples of q."""
    src = os.path.join(ROOT, "paper_2509_12494_amd", "csrc")
    work = tmp_path / "pkg" / "csrc"
    shutil.copytree(src, work)
    shutil.copytree(os.path.join(ROOT, "include"), tmp_path / "include")
    text = (work / "mw_common.h").read_text()
    needle = "(1.0 - 1.0 / (1 << 20))"
    assert needle in text
    (work / "mw_common.h").write_text(text.replace(needle, "(1.0 + 1.0 / (1 << 10))"))
    exe = str(tmp_path / "emulate_bad")
    cxx = CLANG if os.path.exists(CLANG) else shutil.which("clang++")
    subprocess.run([cxx, "-O2", "-std=c++17", "-I" + os.path.join(HERE, "stub"), "-I" + str(work),
                    "-I" + os.path.join(ROOT, "include"), os.path.join(HERE, "emulate.cpp"), "-o", exe], check=True)
    q = W.find_prime(124, 1425)
    xs = [k * q - d for k in range(1, 16) for d in (1, 2, 1 << 20)]
    got = _run(exe, [f"canon 4 {_h(q)} {_h(x)}" for x in xs])
    assert any(g[0] != x % q for g, x in zip(got, xs))
