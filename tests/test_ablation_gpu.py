"""Arithmetic variants of the 124-bit butterfly (the GPU analog of the paper's
MQX ablation: products from v_mul_lo_u32 / v_mul_hi_u32 instead of the
widening multiply-add, carries by compare and select instead of the carry
flags, and both): whole outputs of the 2^16-point forward and inverse
transforms against the oracle's digests (tests/golden/paper_scale.json), at
batch 1 and batch 8 and through the allocation-free path, bit-identical to the
native arithmetic, and the plan's restrictions."""
import hashlib
import json
import os

import numpy as np
import pytest

from paper_2509_12494_amd import mwntt
from paper_2509_12494_amd import workloads as W

from .gpu_util import announce, dev, require_gpu

pytestmark = pytest.mark.gpu

FIXTURE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_scale.json")
VARIANTS = {"mulhi": mwntt.NTT_ARITH_MULHI, "cmpcarry": mwntt.NTT_ARITH_CMPCARRY,
            "plain": mwntt.NTT_ARITH_MULHI | mwntt.NTT_ARITH_CMPCARRY}


def _sha_device(t):
    return hashlib.sha256(np.ascontiguousarray(mwntt.to_host(t).reshape(-1, 2)).astype("<u8").tobytes()).hexdigest()


def _case(name):
    with open(FIXTURE) as f:
        c = json.load(f)["transforms"][name]
    q = W.find_prime(c["bits"], c["prime_seed"])
    A = W.uniform_residues(W.rng(c["input_seed"]), q, 1 << c["log2n"], 2)
    return c, q, A


@pytest.mark.parametrize("variant", sorted(VARIANTS))
@pytest.mark.parametrize("name", ["fwd_2e16_124bit", "inv_2e16_124bit"])
def test_variant_whole_output(name, variant):
    require_gpu()
    import torch
    c, q, A = _case(name)
    inverse = c["op"] == "inv"
    plan = mwntt.ntt_plan(16, q, 2, flags=VARIANTS[variant])
    native = mwntt.ntt_plan(16, q, 2)
    n = plan.n
    for batch in (1, 8):
        a = dev(np.tile(A, (batch, 1)))
        out = torch.full_like(a, -1)
        announce("variant", variant, name, batch)
        (plan.inverse if inverse else plan.forward)(out, a, batch=batch)
        torch.cuda.synchronize()
        for i in range(batch):
            assert _sha_device(out[i * n:(i + 1) * n]) == c["output_sha256"], f"{variant} batch {batch} poly {i}"
        outn = torch.full_like(a, -1)
        plan.transform_noalloc(inverse, outn, a, batch=batch)
        torch.cuda.synchronize()
        assert torch.equal(outn, out)
    # random batch: identical to the native arithmetic
    R = dev(W.uniform_residues(W.rng(77), q, 4 * n, 2))
    o1, o2 = torch.empty_like(R), torch.empty_like(R)
    (plan.inverse if inverse else plan.forward)(o1, R, batch=4)
    (native.inverse if inverse else native.forward)(o2, R, batch=4)
    torch.cuda.synchronize()
    assert torch.equal(o1, o2)
    plan.destroy()
    native.destroy()


def test_variant_plan_restrictions():
    require_gpu()
    import torch
    q124 = W.find_prime(124, 2001)
    q60 = W.find_prime(60, 2001)
    for bad in ((15, q124, 2), (16, q60, 1), (17, q124, 2)):
        with pytest.raises(mwntt.MwError) as e:
            mwntt.ntt_plan(*bad, flags=mwntt.NTT_ARITH_MULHI)
        assert e.value.status == -1
    plan = mwntt.ntt_plan(16, q124, 2, flags=mwntt.NTT_ARITH_CMPCARRY)
    with pytest.raises(mwntt.MwError):
        plan.split = 6
    with pytest.raises(mwntt.MwError):
        plan.set_tiles(1, 1, 1)
    x = torch.zeros(plan.n, 2, dtype=torch.int64, device="cuda")
    with pytest.raises(mwntt.MwError):
        mwntt.NttBatch([(plan, mwntt.NTT_JOB_FORWARD, x, None, x)])
    plan.destroy()
