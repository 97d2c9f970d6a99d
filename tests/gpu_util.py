"""Helpers shared by the GPU parity tests (device transfer, seeded inputs)."""
import functools
import sys

import numpy as np

from paper_2509_12494_amd import mwntt
from paper_2509_12494_amd import workloads as W


def require_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a visible GPU"
    mwntt.lib()       # the HIP library must load; there is no fallback


def announce(*parts):
    """Name the case on stdout before it touches the GPU."""
    print("[case]", *parts, flush=True)
    sys.stdout.flush()


def dev(arr):
    return mwntt.to_device(arr)


def host_ints(t, limbs):
    return W.to_ints(mwntt.to_host(t).reshape(-1, limbs))


def edge_values(q):
    return [0, 1, 2, 3, q - 1, q - 2, q - 3, q // 2, (q + 1) // 2, q >> 1 | 1,
            (1 << 64) % q, ((1 << 64) - 1) % q, ((1 << 32) + 7) % q]


@functools.lru_cache(maxsize=None)
def prime(bits, seed):
    return W.find_prime(bits, seed)


def bitrev(x, bits):
    r = 0
    for _ in range(bits):
        r = (r << 1) | (x & 1)
        x >>= 1
    return r
