"""Whole-output parity at paper scale, element by element, against the CPU
oracle (the paper's standard is results bitwise identical to a reference
library, Evaluation; here the reference is the oracle's definition).

tests/golden/paper_scale.json holds, per case, the SHA-256 of the oracle's
whole canonical output (written by tests/golden/make_digests.py from
oracle.ntt.forward_at / inverse_at, O(N) per output index, and the oracle's
schoolbook negacyclic product) and 64 sampled values to localise a mismatch.
Each GPU configuration that a benchmark figure comes from is tied to these:

* plain transforms at 2^16 and 2^17 (124- and 60-bit, forward and inverse; 252-bit
  forward at 2^16) in the single-transform (latency) configuration and in the
  large-batch (throughput) configuration (the input replicated; the test asserts
  which configuration ran), the allocation-free path, and executor runs of one
  width;
* the fused products of 256 pairs at 2^14 (executor, and replays of a captured
  hipGraph): 8 whole products;
* the mixed 96-polynomial batch (2^12 .. 2^16, 60/124-bit): 64 oracle samples
  of every forward output and 16 of every inverse output.
"""
import functools
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


@functools.lru_cache(maxsize=None)
def _fixture():
    with open(FIXTURE) as f:
        return json.load(f)


def _sha(arr):
    return hashlib.sha256(np.ascontiguousarray(arr, dtype=np.uint64).astype("<u8").tobytes()).hexdigest()


def _sha_device(t, limbs):
    return _sha(mwntt.to_host(t).reshape(-1, limbs))


def _where(got_t, limbs, samples):
    """First sampled index where the device output differs from the oracle."""
    got = W.to_ints(mwntt.to_host(got_t).reshape(-1, limbs))
    for k, v in sorted(samples.items(), key=lambda kv: int(kv[0])):
        if got[int(k)] != int(v):
            return f"index {k}: got {got[int(k)]:#x}, oracle {int(v):#x}"
    return "sampled indices agree; mismatch elsewhere"


# the cases make_digests.py writes (listed here so that a fixture missing a
# case fails its test instead of dropping it from collection)
TRANSFORM_CASES = ["fwd_2e16_124bit", "inv_2e16_124bit", "fwd_2e17_124bit", "inv_2e17_124bit",
                   "fwd_2e16_60bit", "inv_2e16_60bit", "fwd_2e17_60bit", "inv_2e17_60bit", "fwd_2e16_252bit"]


@functools.lru_cache(maxsize=None)
def _transform_input(name):
    c = _fixture()["transforms"][name]
    q = W.find_prime(c["bits"], c["prime_seed"])
    assert str(q) == c["q"]
    limbs = W.limbs_for_bits(c["bits"])
    A = W.uniform_residues(W.rng(c["input_seed"]), q, 1 << c["log2n"], limbs)
    assert _sha(A) == c["input_sha256"], "seeded input differs from the fixture's"
    return c, q, limbs, A


@pytest.mark.parametrize("name", TRANSFORM_CASES)
def test_plain_transform_whole_output(name):
    require_gpu()
    import torch
    c, q, limbs, A = _transform_input(name)
    inverse = c["op"] == "inv"
    plan = mwntt.ntt_plan(c["log2n"], q, limbs)
    n = plan.n
    run = plan.inverse if inverse else plan.forward

    # single-transform (latency) configuration
    assert plan.config_for(1)[0] is False
    a = dev(A)
    out = torch.full_like(a, -1)
    announce("paper scale latency", name)
    run(out, a, batch=1)
    torch.cuda.synchronize()
    assert _sha_device(out, limbs) == c["output_sha256"], _where(out, limbs, c["samples"])

    # large-batch (throughput) configuration: the input replicated
    batch = max(1, (1 << 19) >> c["log2n"])
    large, split = plan.config_for(batch)
    assert large and split, "the throughput configuration was not picked"
    ab = dev(np.tile(A, (batch, 1)))
    outb = torch.full_like(ab, -1)
    announce("paper scale throughput", name, batch, split)
    run(outb, ab, batch=batch)
    torch.cuda.synchronize()
    for i in range(batch):
        assert _sha_device(outb[i * n:(i + 1) * n], limbs) == c["output_sha256"], \
            f"polynomial {i}: " + _where(outb[i * n:(i + 1) * n], limbs, c["samples"])

    # the allocation-free path, same batch
    outn = torch.full_like(ab, -1)
    announce("paper scale noalloc", name, batch)
    plan.transform_noalloc(inverse, outn, ab, batch=batch)
    torch.cuda.synchronize()
    assert torch.equal(outn, outb)

    # the batched executor, one width: `batch` jobs
    outs = [torch.full_like(a, -1) for _ in range(batch)]
    op = mwntt.NTT_JOB_INVERSE if inverse else mwntt.NTT_JOB_FORWARD
    ex = mwntt.NttBatch([(plan, op, ab[i * n:(i + 1) * n], None, outs[i]) for i in range(batch)])
    announce("paper scale executor", name, ex.info())
    ex.run()
    ex.check()
    for i, o in enumerate(outs):
        assert _sha_device(o, limbs) == c["output_sha256"], f"executor job {i}: " + _where(o, limbs, c["samples"])
    ex.destroy()
    plan.destroy()


def test_fused_products_whole_output():
    require_gpu()
    import torch
    fx = _fixture()["fused"]
    q, a, b = W.config_fused()
    assert str(q) == fx["q"]
    pairs, n = a.shape[0], a.shape[1]
    plan = mwntt.ntt_plan(fx["log2n"], q, 2)
    da, db = dev(a.reshape(-1, 2)), dev(b.reshape(-1, 2))
    out = torch.full_like(da, -1)
    ex = mwntt.NttBatch([(plan, mwntt.NTT_JOB_POLYMUL, da[i * n:(i + 1) * n], db[i * n:(i + 1) * n],
                          out[i * n:(i + 1) * n]) for i in range(pairs)])

    def check(tag):
        for p, want in fx["products"].items():
            p = int(p)
            assert _sha(a[p]) == want["a_sha256"] and _sha(b[p]) == want["b_sha256"]
            o = out[p * n:(p + 1) * n]
            assert _sha_device(o, 2) == want["output_sha256"], f"{tag} pair {p}: " + _where(o, 2, want["samples"])

    announce("fused 256 x 2^14", ex.info())
    ex.run()
    ex.check()
    check("eager")
    # hipGraph capture of one run, replayed with eager work in between
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            ex.run(stream=s)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        out.fill_(-1)
        torch.cuda.synchronize()
        announce("fused graph replay", rep)
        g.replay()
        torch.cuda.synchronize()
        check(f"replay {rep}")
    del g
    ex.destroy()
    plan.destroy()


def test_mixed_batch_every_job_sampled():
    require_gpu()
    import torch
    fx = _fixture()["batched"]
    polys = W.config_batched()
    assert len(polys) == fx["count"] == 96
    plans, ins, fwd_out, inv_out = [], [], [], []
    for i, (log2n, q, limbs, coeffs) in enumerate(polys):
        j = fx["jobs"][i]
        assert j["log2n"] == log2n and j["q"] == str(q) and _sha(coeffs) == j["input_sha256"]
        plans.append(mwntt.ntt_plan(log2n, q, limbs))
        ins.append(dev(coeffs))
        fwd_out.append(torch.full_like(ins[-1], -1))
        inv_out.append(torch.full_like(ins[-1], -1))
    for op, outs, key in ((mwntt.NTT_JOB_FORWARD, fwd_out, "fwd"), (mwntt.NTT_JOB_INVERSE, inv_out, "inv")):
        ex = mwntt.NttBatch([(plans[i], op, ins[i], None, outs[i]) for i in range(96)])
        announce("mixed 96", key, ex.info())
        ex.run()
        ex.check()
        for i in range(96):
            limbs = polys[i][2]
            got = W.to_ints(mwntt.to_host(outs[i]).reshape(-1, limbs))
            for k, v in fx["jobs"][i][key].items():
                assert got[int(k)] == int(v), f"{key} job {i} (2^{polys[i][0]}, {limbs} limbs) index {k}"
        ex.destroy()
    for p in plans:
        p.destroy()
