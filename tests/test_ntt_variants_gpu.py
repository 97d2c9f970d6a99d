"""Every decomposition and tile shape gives the same bits (differential test).

A missing barrier or a wrong LDS index in one tile shape shows up as a
difference from the oracle in that shape only, so each shape is compared
against the oracle's transform on the same seeded input."""
import functools

import pytest

import oracle
from paper_2509_12494_amd import mwntt
from paper_2509_12494_amd import workloads as W

from .gpu_util import announce, dev, host_ints, prime, require_gpu

pytestmark = pytest.mark.gpu


@functools.lru_cache(maxsize=None)
def _case(bits, log2n):
    q = prime(bits, 31)
    limbs = W.limbs_for_bits(bits)
    A = W.uniform_residues(W.rng(31 + log2n), q, 3 << log2n, limbs)   # 3 transforms
    a = W.to_ints(A)
    n = 1 << log2n
    want = [oracle.ntt.ntt_negacyclic(a[i * n:(i + 1) * n], q) for i in range(3)]
    return q, limbs, A, sum(want, [])


def _shapes(plan, pass_, logl, max_lines):
    out = []
    for logp in range(1, 5):
        for lines in (1, 2, 4, 8, 16, 32):
            if lines > max_lines:
                continue
            try:
                plan.set_tiles(pass_, logp, lines)
            except mwntt.MwError:
                continue
            out.append((logp, lines))
    return out


def _check(plan, A, want, limbs, tag):
    import torch
    x = dev(A)
    y = torch.empty_like(x)
    plan.forward(y, x, batch=3)
    z = torch.empty_like(x)
    plan.inverse(z, y, batch=3)
    torch.cuda.synchronize()
    assert host_ints(y, limbs) == want, tag
    assert torch.equal(z, x), tag


@pytest.mark.parametrize("bits", [60, 124, 252])
@pytest.mark.parametrize("log2n", [5, 8, 10])
def test_full_tile_shapes(log2n, bits):
    require_gpu()
    q, limbs, A, want = _case(bits, log2n)
    plan = mwntt.ntt_plan(log2n, q, limbs)
    shapes = _shapes(plan, plan.PASS_FULL, log2n, 64)
    assert shapes
    for logp, lines in shapes:
        announce("full shape", log2n, bits, logp, lines)
        plan.set_tiles(plan.PASS_FULL, logp, lines)
        _check(plan, A, want, limbs, (logp, lines))
    plan.destroy()


@pytest.mark.parametrize("bits", [60, 124, 252])
@pytest.mark.parametrize("log2n,log_n1", [(8, 4), (10, 3), (10, 5), (10, 7), (11, 5)])
def test_two_pass_shapes(log2n, log_n1, bits):
    require_gpu()
    q, limbs, A, want = _case(bits, log2n)
    plan = mwntt.ntt_plan(log2n, q, limbs)
    plan.split = log_n1
    log_n2 = log2n - log_n1
    col = _shapes(plan, plan.PASS_COL, log_n1, 1 << log_n2)
    plan.split = log_n1
    row = _shapes(plan, plan.PASS_ROW, log_n2, 1 << log_n1)
    assert col and row
    plan.split = log_n1
    d_col, d_row = plan.get_tiles(plan.PASS_COL), plan.get_tiles(plan.PASS_ROW)
    for logp, lines in col:
        announce("col shape", log2n, log_n1, bits, logp, lines)
        plan.set_tiles(plan.PASS_COL, logp, lines)
        plan.set_tiles(plan.PASS_ROW, *d_row)
        _check(plan, A, want, limbs, ("col", logp, lines))
    plan.set_tiles(plan.PASS_COL, *d_col)
    for logp, lines in row:
        announce("row shape", log2n, log_n1, bits, logp, lines)
        plan.set_tiles(plan.PASS_ROW, logp, lines)
        _check(plan, A, want, limbs, ("row", logp, lines))
    plan.destroy()
