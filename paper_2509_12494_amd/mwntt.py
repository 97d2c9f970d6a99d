"""Python binding of libmwntt.so (ctypes): argument marshalling only.

Every function here forwards to the C ABI declared in include/mwntt.h; the
arithmetic runs in the library's HIP kernels.  There is no CPU fallback: if the
library is missing, importing the functions raises.

Device buffers are torch tensors (any integer dtype, contiguous, on the GPU)
holding `limbs` little-endian 64-bit words per residue, or raw device pointers
(ints).  Moduli, roots and scalars are Python ints.  ``stream`` defaults to
torch's current stream.
"""
from __future__ import annotations

import atexit
import ctypes
import functools
import os
import weakref
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
# MWNTT_LIB loads another build of the library instead (the host-sanitizer
# builds of `python -m paper_2509_12494_amd.build --sanitize ...`).
LIB_PATH = os.environ.get("MWNTT_LIB") or os.path.join(HERE, "libmwntt.so")

MW_OK = 0
NTT_BITREV_OUT = 0x1
NTT_BITREV_IN = 0x2
NTT_ARITH_MULHI = 0x10
NTT_ARITH_CMPCARRY = 0x20

NTT_JOB_FORWARD = 0
NTT_JOB_INVERSE = 1
NTT_JOB_POLYMUL = 2

_lib = None

try:
    # direct-call shim for the hot entry points (csrc/mw_pycall.c, built with
    # the library): the same calls into libmwntt as through ctypes, with less
    # per-call marshalling; without it the ctypes path below is used
    from . import _mwcall
except ImportError:
    _mwcall = None

_HOT = ("ntt_forward", "ntt_inverse", "vec_addmod", "vec_submod", "vec_mulmod", "vec_axpymod")
_BLAS_OP = {"vec_addmod": 0, "vec_submod": 1, "vec_mulmod": 2}


class NttJob(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("op", ctypes.c_uint32), ("in_", ctypes.c_void_p),
                ("in2", ctypes.c_void_p), ("out", ctypes.c_void_p)]


MW_REQ_NTT_FORWARD, MW_REQ_NTT_INVERSE, MW_REQ_POLYMUL = 0, 1, 2
MW_REQ_VEC_ADDMOD, MW_REQ_VEC_SUBMOD, MW_REQ_VEC_MULMOD, MW_REQ_VEC_AXPYMOD = 3, 4, 5, 6
MW_EBUSY = -7
MW_ENONCANON = -8


class MwRequest(ctypes.Structure):
    _fields_ = [("op", ctypes.c_uint32), ("plan", ctypes.c_void_p), ("q", ctypes.c_uint64 * 4),
                ("limbs", ctypes.c_uint32), ("alpha", ctypes.c_uint64 * 4), ("n", ctypes.c_uint64),
                ("in_", ctypes.c_void_p), ("in2", ctypes.c_void_p)]


class MwServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("max_inflight", ctypes.c_uint32),
                ("max_batch", ctypes.c_uint32), ("dry_run", ctypes.c_uint32), ("spin_us", ctypes.c_uint32),
                ("resident", ctypes.c_uint32), ("resident_max_tiles", ctypes.c_uint32),
                ("resident_wait_us", ctypes.c_uint32)]


class MwServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("batches", ctypes.c_uint64),
                ("max_batch_seen", ctypes.c_uint64), ("queue_peak", ctypes.c_uint64),
                ("inflight_peak", ctypes.c_uint64), ("pool_peak", ctypes.c_size_t),
                ("resident_requests", ctypes.c_uint64), ("resident_launches", ctypes.c_uint64),
                ("resident_yields", ctypes.c_uint64)]


class MwError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_str(status)} ({status})")


def lib() -> ctypes.CDLL:
    """Load libmwntt.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2509_12494_amd.build` (or __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    vp, u32, u64p, sz = ctypes.c_void_p, ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint64), ctypes.c_size_t
    sig = {
        "mw_status_str": (ctypes.c_char_p, [ctypes.c_int]),
        "mw_version": (ctypes.c_char_p, []),
        "vec_addmod": (ctypes.c_int, [vp, vp, vp, sz, u64p, u32, vp]),
        "vec_submod": (ctypes.c_int, [vp, vp, vp, sz, u64p, u32, vp]),
        "vec_mulmod": (ctypes.c_int, [vp, vp, vp, sz, u64p, u32, vp]),
        "vec_axpymod": (ctypes.c_int, [vp, u64p, vp, sz, u64p, u32, vp]),
        "ntt_plan": (ctypes.c_int, [ctypes.POINTER(vp), u32, u64p, u32, u64p, u32]),
        "ntt_plan_destroy": (ctypes.c_int, [vp]),
        "ntt_plan_root": (ctypes.c_int, [vp, u64p]),
        "ntt_plan_set_split": (ctypes.c_int, [vp, u32]),
        "ntt_plan_get_split": (ctypes.c_int, [vp, ctypes.POINTER(u32)]),
        "ntt_plan_set_tiles": (ctypes.c_int, [vp, u32, u32, u32]),
        "ntt_plan_get_tiles": (ctypes.c_int, [vp, u32, ctypes.POINTER(u32), ctypes.POINTER(u32)]),
        "ntt_forward": (ctypes.c_int, [vp, vp, vp, u32, vp]),
        "ntt_forward_pass": (ctypes.c_int, [vp, u32, vp, vp, u32, vp]),
        "ntt_inverse": (ctypes.c_int, [vp, vp, vp, u32, vp]),
        "ntt_transform_noalloc": (ctypes.c_int, [vp, u32, vp, vp, u32, vp]),
        "ntt_plan_config_for": (ctypes.c_int, [vp, u32, ctypes.POINTER(u32), ctypes.POINTER(u32)]),
        "ntt_batch_create": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.POINTER(NttJob), u32]),
        "ntt_batch_run": (ctypes.c_int, [vp, vp]),
        "ntt_batch_info": (ctypes.c_int, [vp, ctypes.POINTER(u32), ctypes.POINTER(u32)]),
        "ntt_batch_check": (ctypes.c_int, [vp]),
        "ntt_batch_destroy": (ctypes.c_int, [vp]),
        "mw_server_create": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.POINTER(MwServerConfig)]),
        "mw_server_submit": (ctypes.c_int, [vp, ctypes.POINTER(MwRequest), ctypes.POINTER(ctypes.c_uint64)]),
        "mw_server_result": (ctypes.c_int, [vp, ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(vp),
                                            ctypes.POINTER(ctypes.c_double)]),
        "mw_server_release": (ctypes.c_int, [vp, ctypes.c_uint64]),
        "mw_server_drain": (ctypes.c_int, [vp]),
        "mw_server_get_stats": (ctypes.c_int, [vp, ctypes.POINTER(MwServerStats)]),
        "mw_server_replay": (ctypes.c_int, [vp, ctypes.POINTER(MwRequest), ctypes.POINTER(ctypes.c_double), u32,
                                            ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
        "mw_server_destroy": (ctypes.c_int, [vp]),
        "mw_copy": (ctypes.c_int, [vp, vp, sz, vp]),
        "mw_canonical_root": (ctypes.c_int, [u64p, u32, u32, u64p]),
        "mw_shoup_companion": (ctypes.c_int, [u64p, u64p, u32, u64p]),
        "mw_barrett_mu": (ctypes.c_int, [u64p, u32, u64p]),
        "vec_mulmod_set_product": (ctypes.c_int, [u32, u32]),
        "vec_mulmod_get_product": (ctypes.c_int, [u32, ctypes.POINTER(u32)]),
        "mw_set_validate": (ctypes.c_int, [ctypes.c_int]),
        "mw_get_validate": (ctypes.c_int, []),
        "mw_check": (ctypes.c_int, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    if _mwcall is not None:
        _mwcall.bind(*(ctypes.cast(getattr(L, n), ctypes.c_void_p).value for n in _HOT))
    _lib = L
    return L


def status_str(status: int) -> str:
    return lib().mw_status_str(status).decode()


def version() -> str:
    return lib().mw_version().decode()


def _check(status: int, where: str) -> None:
    if status != MW_OK:
        raise MwError(status, where)


@functools.lru_cache(maxsize=1024)
def _words(x: int, limbs: int, size: int = 4):
    """`limbs` little-endian 64-bit words of x in a ctypes array of `size` words.

    Cached: the arrays are read-only inputs of the C calls (moduli, roots and
    scalars recur on every call), so they are built once per value."""
    if limbs > size:
        raise ValueError(f"at most {size} words here")
    if x < 0 or x >= 1 << (64 * limbs):
        raise ValueError("value does not fit the limb count")
    arr = (ctypes.c_uint64 * size)()
    for i in range(limbs):
        arr[i] = (x >> (64 * i)) & (2**64 - 1)
    return arr


@functools.lru_cache(maxsize=1024)
def _words_ref(x: int, limbs: int):
    """(array, address) of _words(x, limbs), for the direct-call shim; the
    caller holds the tuple while the call runs."""
    arr = _words(x, limbs)
    return arr, ctypes.addressof(arr)


def _from_words(arr, limbs: int) -> int:
    return sum(int(arr[i]) << (64 * i) for i in range(limbs))


def _ptr(t) -> int:
    if isinstance(t, int):
        return t
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _count(t, limbs: int, n: Optional[int]) -> int:
    if n is not None:
        return n
    if isinstance(t, int):
        raise ValueError("n is required with raw pointers")
    return t.numel() * t.element_size() // (8 * limbs)


# ---------------------------------------------------------------------------
# BLAS
# ---------------------------------------------------------------------------
def _blas(name, c, a, b, q, limbs, n, stream):
    n = _count(c, limbs, n)
    L = lib()
    if _mwcall is not None:
        qref = _words_ref(q, limbs)
        st = _mwcall.blas(_BLAS_OP[name], _ptr(c), _ptr(a), _ptr(b), n, qref[1], limbs, _stream(stream))
    else:
        st = getattr(L, name)(_ptr(c), _ptr(a), _ptr(b), n, _words(q, limbs), limbs, _stream(stream))
    _check(st, name)


def vec_addmod(c, a, b, q: int, limbs: int, n: Optional[int] = None, stream=None) -> None:
    _blas("vec_addmod", c, a, b, q, limbs, n, stream)


def vec_submod(c, a, b, q: int, limbs: int, n: Optional[int] = None, stream=None) -> None:
    _blas("vec_submod", c, a, b, q, limbs, n, stream)


def vec_mulmod(c, a, b, q: int, limbs: int, n: Optional[int] = None, stream=None) -> None:
    _blas("vec_mulmod", c, a, b, q, limbs, n, stream)


def vec_axpymod(y, alpha: int, x, q: int, limbs: int, n: Optional[int] = None, stream=None) -> None:
    n = _count(y, limbs, n)
    L = lib()
    if _mwcall is not None:
        aref, qref = _words_ref(alpha, limbs), _words_ref(q, limbs)
        st = _mwcall.axpy(_ptr(y), aref[1], _ptr(x), n, qref[1], limbs, _stream(stream))
    else:
        st = L.vec_axpymod(_ptr(y), _words(alpha, limbs), _ptr(x), n, _words(q, limbs), limbs, _stream(stream))
    _check(st, "vec_axpymod")


# ---------------------------------------------------------------------------
# NTT
# ---------------------------------------------------------------------------
class NttPlan:
    """Owning wrapper of an ntt_plan_t."""

    def __init__(self, log2n: int, q: int, limbs: int, psi: Optional[int] = None, flags: int = 0):
        self.log2n, self.q, self.limbs, self.flags = log2n, q, limbs, flags
        h = ctypes.c_void_p()
        psi_w = _words(psi, limbs) if psi is not None else None
        _check(lib().ntt_plan(ctypes.byref(h), log2n, _words(q, limbs), limbs, psi_w, flags), "ntt_plan")
        self._h = h

    @property
    def n(self) -> int:
        return 1 << self.log2n

    @property
    def root(self) -> int:
        out = (ctypes.c_uint64 * 4)()
        _check(lib().ntt_plan_root(self._h, out), "ntt_plan_root")
        return _from_words(out, self.limbs)

    @property
    def split(self) -> int:
        v = ctypes.c_uint32()
        _check(lib().ntt_plan_get_split(self._h, ctypes.byref(v)), "ntt_plan_get_split")
        return v.value

    @split.setter
    def split(self, log_n1: int) -> None:
        _check(lib().ntt_plan_set_split(self._h, log_n1), "ntt_plan_set_split")

    PASS_FULL, PASS_COL, PASS_ROW = 0, 1, 2

    def set_tiles(self, pass_: int, log_p: int, lines: int) -> None:
        _check(lib().ntt_plan_set_tiles(self._h, pass_, log_p, lines), "ntt_plan_set_tiles")

    def get_tiles(self, pass_: int):
        lp, ln = ctypes.c_uint32(), ctypes.c_uint32()
        _check(lib().ntt_plan_get_tiles(self._h, pass_, ctypes.byref(lp), ctypes.byref(ln)), "ntt_plan_get_tiles")
        return lp.value, ln.value

    def config_for(self, batch: int):
        """(large-batch configuration?, log2 N1) of a call with `batch` transforms."""
        lg, l1 = ctypes.c_uint32(), ctypes.c_uint32()
        _check(lib().ntt_plan_config_for(self._h, batch, ctypes.byref(lg), ctypes.byref(l1)), "ntt_plan_config_for")
        return bool(lg.value), l1.value

    def _batch(self, t, batch):
        if batch is not None:
            return batch
        if isinstance(t, int):
            raise ValueError("batch is required with raw pointers")
        return t.numel() * t.element_size() // (8 * self.limbs * self.n)

    def forward(self, out, inp, batch: Optional[int] = None, stream=None) -> None:
        b = self._batch(inp, batch)
        L = lib()
        if _mwcall is not None:
            hv = self._h.value if self._h is not None else None
            st = _mwcall.ntt(0, hv, _ptr(out), _ptr(inp), b, _stream(stream))
        else:
            st = L.ntt_forward(self._h, _ptr(out), _ptr(inp), b, _stream(stream))
        _check(st, "ntt_forward")

    def forward_pass(self, pass_: int, out, inp, batch: int, stream=None) -> None:
        """Pass 1 (column tiles, inp -> plan scratch) or 2 (row tiles, scratch -> out)."""
        o = _ptr(out) if out is not None else None
        i = _ptr(inp) if inp is not None else None
        _check(lib().ntt_forward_pass(self._h, pass_, o, i, batch, _stream(stream)), "ntt_forward_pass")

    def inverse(self, out, inp, batch: Optional[int] = None, stream=None) -> None:
        b = self._batch(inp, batch)
        L = lib()
        if _mwcall is not None:
            hv = self._h.value if self._h is not None else None
            st = _mwcall.ntt(1, hv, _ptr(out), _ptr(inp), b, _stream(stream))
        else:
            st = L.ntt_inverse(self._h, _ptr(out), _ptr(inp), b, _stream(stream))
        _check(st, "ntt_inverse")

    def transform_noalloc(self, inverse: bool, out, inp, batch: Optional[int] = None, stream=None) -> None:
        """ntt_transform_noalloc: forward or inverse with the library's static scratch (no allocation)."""
        b = self._batch(inp, batch)
        _check(lib().ntt_transform_noalloc(self._h, 1 if inverse else 0, _ptr(out), _ptr(inp), b, _stream(stream)),
               "ntt_transform_noalloc")

    def destroy(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(lib().ntt_plan_destroy(self._h), "ntt_plan_destroy")
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def ntt_plan(log2n: int, q: int, limbs: int, psi: Optional[int] = None, flags: int = 0) -> NttPlan:
    return NttPlan(log2n, q, limbs, psi, flags)


class NttBatch:
    """Owning wrapper of an ntt_batch_t: many jobs, one launch per phase per run.

    jobs: iterable of (plan, op, inp, inp2, out) with op one of NTT_JOB_*; inp2
    is None except for NTT_JOB_POLYMUL.  The wrapper keeps references to the
    plans and buffers so they outlive the batch."""

    def __init__(self, jobs):
        jobs = list(jobs)
        arr = (NttJob * len(jobs))()
        for i, (plan, op, inp, inp2, out) in enumerate(jobs):
            arr[i].plan = plan._h.value
            arr[i].op = op
            arr[i].in_ = _ptr(inp)
            arr[i].in2 = _ptr(inp2) if inp2 is not None else None
            arr[i].out = _ptr(out)
        h = ctypes.c_void_p()
        _check(lib().ntt_batch_create(ctypes.byref(h), arr, len(jobs)), "ntt_batch_create")
        self._h = h
        self._keep = jobs

    def run(self, stream=None) -> None:
        _check(lib().ntt_batch_run(self._h, _stream(stream)), "ntt_batch_run")

    def check(self) -> None:
        """Synchronize and raise if a run failed inside the kernel."""
        _check(lib().ntt_batch_check(self._h), "ntt_batch_check")

    def info(self):
        t, w = ctypes.c_uint32(), ctypes.c_uint32()
        _check(lib().ntt_batch_info(self._h, ctypes.byref(t), ctypes.byref(w)), "ntt_batch_info")
        return {"tiles": t.value, "launches": w.value}

    def destroy(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(lib().ntt_batch_destroy(self._h), "ntt_batch_destroy")
            self._h = None
            self._keep = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# serving runtime
# ---------------------------------------------------------------------------
def make_request(op: int, inp, inp2=None, plan: Optional[NttPlan] = None, q: int = 0, limbs: int = 0,
                 n: int = 0, alpha: int = 0) -> MwRequest:
    r = MwRequest()
    r.op = op
    r.plan = plan._h.value if plan is not None else None
    if plan is None:
        r.q = _words(q, limbs)
        r.alpha = _words(alpha, limbs)
        r.limbs = limbs
        r.n = n
    r.in_ = _ptr(inp)
    r.in2 = _ptr(inp2) if inp2 is not None else None
    return r


# Servers still alive when the interpreter exits are destroyed first: each
# owns a scheduler thread and possibly a running resident loop.
_live_servers: "weakref.WeakSet[MwServer]" = weakref.WeakSet()


@atexit.register
def _destroy_live_servers() -> None:
    for srv in list(_live_servers):
        try:
            srv.destroy()
        except Exception:
            pass


class MwServer:
    """Owning wrapper of an mw_server_t (continuous batching of NTT / BLAS requests)."""

    def __init__(self, hbm_budget: int, max_inflight: int = 4, max_batch: int = 64, dry_run: bool = False,
                 spin_us: int = 0, resident: bool = False, resident_max_tiles: int = 0,
                 resident_wait_us: int = 0):
        cfg = MwServerConfig(hbm_budget, max_inflight, max_batch, 1 if dry_run else 0, spin_us,
                             1 if resident else 0, resident_max_tiles, resident_wait_us)
        h = ctypes.c_void_p()
        _check(lib().mw_server_create(ctypes.byref(h), ctypes.byref(cfg)), "mw_server_create")
        self._h = h
        self._keep = {}
        _live_servers.add(self)

    def submit(self, req: MwRequest, keep=None) -> int:
        t = ctypes.c_uint64()
        _check(lib().mw_server_submit(self._h, ctypes.byref(req), ctypes.byref(t)), "mw_server_submit")
        if keep is not None:
            self._keep[t.value] = keep
        return t.value

    def result(self, ticket: int, wait: bool = True):
        """(device pointer of the output or None, latency in us); raises MwError (MW_EBUSY if not ready)."""
        p, lat = ctypes.c_void_p(), ctypes.c_double()
        _check(lib().mw_server_result(self._h, ticket, 1 if wait else 0, ctypes.byref(p), ctypes.byref(lat)),
               "mw_server_result")
        return p.value, lat.value

    def release(self, ticket: int) -> None:
        _check(lib().mw_server_release(self._h, ticket), "mw_server_release")
        self._keep.pop(ticket, None)

    def drain(self) -> None:
        _check(lib().mw_server_drain(self._h), "mw_server_drain")

    def stats(self) -> dict:
        st = MwServerStats()
        _check(lib().mw_server_get_stats(self._h, ctypes.byref(st)), "mw_server_get_stats")
        return {f: getattr(st, f) for f, _ in MwServerStats._fields_}

    def replay(self, reqs, arrival_us):
        """Open-loop replay; returns (latencies in us, makespan in us)."""
        n = len(reqs)
        arr = (MwRequest * n)(*reqs)
        arrivals = (ctypes.c_double * n)(*arrival_us)
        lat = (ctypes.c_double * n)()
        span = ctypes.c_double()
        _check(lib().mw_server_replay(self._h, arr, arrivals, n, lat, ctypes.byref(span)), "mw_server_replay")
        return list(lat), span.value

    def destroy(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(lib().mw_server_destroy(self._h), "mw_server_destroy")
            self._h = None
            self._keep = {}

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def copy_to_tensor(ptr: int, like, stream=None):
    """Copy a server-owned device buffer into a new device tensor shaped like `like`."""
    import torch
    out = torch.empty_like(like)
    nbytes = out.numel() * out.element_size()
    _check(lib().mw_copy(out.data_ptr(), ptr, nbytes, _stream(stream)), "mw_copy")
    return out


def set_mulmod_product(limbs: int, karatsuba: bool) -> None:
    """vec_mulmod's full product for one width: Karatsuba (Eq. mulk) or schoolbook."""
    _check(lib().vec_mulmod_set_product(limbs, 1 if karatsuba else 0), "vec_mulmod_set_product")


def get_mulmod_product(limbs: int) -> bool:
    k = ctypes.c_uint32()
    _check(lib().vec_mulmod_get_product(limbs, ctypes.byref(k)), "vec_mulmod_get_product")
    return bool(k.value)


# ---------------------------------------------------------------------------
# validate mode (input canonicality checks)
# ---------------------------------------------------------------------------
def set_validate(on: bool) -> None:
    _check(lib().mw_set_validate(1 if on else 0), "mw_set_validate")


def get_validate() -> bool:
    return bool(lib().mw_get_validate())


def check(stream=None) -> None:
    """Synchronizes the stream; raises MwError(MW_ENONCANON) if a checked input was not canonical."""
    _check(lib().mw_check(_stream(stream)), "mw_check")


# ---------------------------------------------------------------------------
# host-only helpers
# ---------------------------------------------------------------------------
def canonical_root(q: int, limbs: int, log2n: int) -> int:
    out = (ctypes.c_uint64 * 4)()
    _check(lib().mw_canonical_root(_words(q, limbs), limbs, log2n, out), "mw_canonical_root")
    return _from_words(out, limbs)


def shoup_companion(w: int, q: int, limbs: int) -> int:
    out = (ctypes.c_uint64 * 4)()
    _check(lib().mw_shoup_companion(_words(w, limbs), _words(q, limbs), limbs, out), "mw_shoup_companion")
    return _from_words(out, limbs)


def barrett_mu(q: int, limbs: int) -> int:
    out = (ctypes.c_uint64 * 4)()
    _check(lib().mw_barrett_mu(_words(q, limbs), limbs, out), "mw_barrett_mu")
    return _from_words(out, limbs)


# ---------------------------------------------------------------------------
# tensor helpers (layout only)
# ---------------------------------------------------------------------------
def to_device(arr, device="cuda"):
    """(n, limbs) uint64 numpy array -> int64 torch tensor on the device."""
    import numpy as np
    import torch
    a = np.ascontiguousarray(arr, dtype=np.uint64)
    return torch.from_numpy(a.view(np.int64)).to(device)


def to_host(t):
    """int64 torch tensor -> uint64 numpy array of the same shape."""
    import numpy as np
    return t.detach().cpu().numpy().view(np.uint64)
