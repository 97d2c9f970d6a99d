"""Plain scalar C++ CPU baseline of the hot path (negacyclic NTT and modular
BLAS with unsigned __int128 double-words, schoolbook products and Barrett
reduction), timed beside the GPU.  `build()` compiles cpu_ref.cpp with g++
into libcpuref.so next to it; the functions below marshal numpy arrays of
uint64 words (n x limbs, little-endian words) to its C entry points.

Nothing in the GPU library uses this module: it is a measured baseline.

The library is built for x86-64-v3 (AVX2, BMI2; no intrinsics in the source)
rather than -march=native, because it is built on one machine and timed on
another (the GPU host)."""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cpu_ref.cpp")
LIB = os.path.join(HERE, "libcpuref.so")
FLAGS = ["-O3", "-march=x86-64-v3", "-std=c++17", "-fPIC", "-shared", "-pthread", "-Wall", "-Wextra"]

STATUS = {0: "ok", -1: "invalid argument", -2: "modulus outside its class or q != 1 mod 2N",
          -3: "out of memory", -4: "no primitive 2N-th root"}
OPS = {"add": 0, "sub": 1, "mul": 2, "axpy": 3}

_lib = None


def build(verbose: bool = False) -> None:
    cmd = ["g++"] + FLAGS + ["-o", LIB + ".tmp", SRC]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError(f"{LIB} is not built: run __graft_entry__.build()")
        L = ctypes.CDLL(LIB)
        vp, u32, u64p = ctypes.c_void_p, ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint64)
        L.cpuref_plan_create.argtypes = [ctypes.POINTER(vp), u32, u64p, u32, u64p]
        L.cpuref_plan_root.argtypes = [vp, u64p]
        L.cpuref_plan_destroy.argtypes = [vp]
        L.cpuref_ntt.argtypes = [vp, u64p, u64p, u32, u32, u32]
        L.cpuref_blas.argtypes = [u32, u64p, u64p, u64p, ctypes.c_uint64, u64p, u32, u64p, u32]
        for f in (L.cpuref_plan_create, L.cpuref_plan_root, L.cpuref_plan_destroy, L.cpuref_ntt, L.cpuref_blas):
            f.restype = ctypes.c_int
        _lib = L
    return _lib


def _check(st: int, where: str) -> None:
    if st != 0:
        raise RuntimeError(f"{where}: {STATUS.get(st, st)} ({st})")


def _words(x: int, limbs: int):
    return (ctypes.c_uint64 * limbs)(*[(x >> (64 * i)) & ((1 << 64) - 1) for i in range(limbs)])


def _ptr(a: np.ndarray):
    assert a.dtype == np.uint64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


class Plan:
    """Tables of one transform size and modulus (psi: None for the smallest
    primitive 2N-th root)."""

    def __init__(self, log2n: int, q: int, limbs: int, psi=None):
        h = ctypes.c_void_p()
        _check(lib().cpuref_plan_create(ctypes.byref(h), log2n, _words(q, limbs), limbs,
                                        _words(psi, limbs) if psi is not None else None), "cpuref_plan_create")
        self._h, self.log2n, self.q, self.limbs = h, log2n, q, limbs

    def root(self) -> int:
        w = (ctypes.c_uint64 * self.limbs)()
        _check(lib().cpuref_plan_root(self._h, w), "cpuref_plan_root")
        return sum(int(w[i]) << (64 * i) for i in range(self.limbs))

    def transform(self, data: np.ndarray, inverse: bool = False, threads: int = 1) -> np.ndarray:
        """Transforms a (batch * N, limbs) array; returns a new array."""
        n = 1 << self.log2n
        src = np.ascontiguousarray(data, dtype=np.uint64).reshape(-1, self.limbs)
        assert src.shape[0] % n == 0
        out = np.empty_like(src)
        _check(lib().cpuref_ntt(self._h, _ptr(out), _ptr(src), src.shape[0] // n, 1 if inverse else 0, threads),
               "cpuref_ntt")
        return out

    def destroy(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().cpuref_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def blas(op: str, a: np.ndarray, b: np.ndarray, q: int, limbs: int, alpha: int = 0, threads: int = 1) -> np.ndarray:
    """c = a op b (axpy: c = alpha*a + b) over (n, limbs) arrays."""
    a = np.ascontiguousarray(a, dtype=np.uint64).reshape(-1, limbs)
    b = np.ascontiguousarray(b, dtype=np.uint64).reshape(-1, limbs)
    assert a.shape == b.shape
    c = np.empty_like(a)
    _check(lib().cpuref_blas(OPS[op], _ptr(c), _ptr(a), _ptr(b), a.shape[0], _words(q, limbs), limbs,
                             _words(alpha, limbs) if op == "axpy" else None, threads), "cpuref_blas")
    return c
