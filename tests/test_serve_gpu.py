"""Serving runtime on the GPU: every result in a mixed, batched, overlapping
stream is bit-identical to the same operation run alone through the plain
entry points (and to the oracle on sampled outputs), also when a small HBM
budget forces queueing and when 60-, 124- and 252-bit requests are mixed; an
open-loop Poisson replay completes every request."""
import pytest

import oracle
from paper_2509_12494_amd import mwntt
from paper_2509_12494_amd import workloads as W

from .gpu_util import announce, dev, host_ints, prime, require_gpu

pytestmark = pytest.mark.gpu

OPS = [mwntt.MW_REQ_NTT_FORWARD, mwntt.MW_REQ_NTT_INVERSE, mwntt.MW_REQ_POLYMUL,
       mwntt.MW_REQ_VEC_MULMOD, mwntt.MW_REQ_VEC_AXPYMOD, mwntt.MW_REQ_VEC_ADDMOD, mwntt.MW_REQ_VEC_SUBMOD]


def _workload(count, seed, log2_range=(10, 13), wide=False, widths=None):
    import torch
    g = W.rng(seed)
    plans = {}
    items = []
    for i in range(count):
        op = OPS[i % len(OPS)]
        if widths:
            bits = widths[int(g.integers(0, len(widths)))]
        else:
            bits = [60, 124, 252][int(g.integers(0, 3))] if wide else (60 if g.random() < 0.5 else 124)
        q = prime(bits, 61 + (i % 2))
        limbs = W.limbs_for_bits(bits)
        if op <= mwntt.MW_REQ_POLYMUL:
            log2n = int(g.integers(log2_range[0], log2_range[1] + 1))
            n = 1 << log2n
            if (log2n, q) not in plans:
                plans[(log2n, q)] = mwntt.ntt_plan(log2n, q, limbs)
            plan = plans[(log2n, q)]
        else:
            n = int(2.0 ** g.uniform(log2_range[0], log2_range[1]))
            plan = None
        A = W.uniform_residues(g, q, n, limbs)
        B = W.uniform_residues(g, q, n, limbs)
        alpha = W.uniform_scalar(g, q, limbs)
        items.append(dict(op=op, q=q, limbs=limbs, n=n, plan=plan, A=A, B=B, a=dev(A), b=dev(B), alpha=alpha))
    return items, plans


def _request(it):
    needs_b = it["op"] != mwntt.MW_REQ_NTT_FORWARD and it["op"] != mwntt.MW_REQ_NTT_INVERSE
    if it["plan"] is not None:
        return mwntt.make_request(it["op"], it["a"], it["b"] if needs_b else None, plan=it["plan"])
    return mwntt.make_request(it["op"], it["a"], it["b"], q=it["q"], limbs=it["limbs"], n=it["n"], alpha=it["alpha"])


def _alone(it):
    """The same operation through the plain entry points."""
    import torch
    a, b, q, limbs, plan = it["a"], it["b"], it["q"], it["limbs"], it["plan"]
    out = torch.empty_like(a)
    op = it["op"]
    if op == mwntt.MW_REQ_NTT_FORWARD:
        plan.forward(out, a)
    elif op == mwntt.MW_REQ_NTT_INVERSE:
        plan.inverse(out, a)
    elif op == mwntt.MW_REQ_POLYMUL:
        fa, fb = torch.empty_like(a), torch.empty_like(b)
        plan.forward(fa, a)
        plan.forward(fb, b)
        mwntt.vec_mulmod(fa, fa, fb, q, limbs)
        plan.inverse(out, fa)
    elif op == mwntt.MW_REQ_VEC_MULMOD:
        mwntt.vec_mulmod(out, a, b, q, limbs)
    elif op == mwntt.MW_REQ_VEC_ADDMOD:
        mwntt.vec_addmod(out, a, b, q, limbs)
    elif op == mwntt.MW_REQ_VEC_SUBMOD:
        mwntt.vec_submod(out, a, b, q, limbs)
    else:
        out.copy_(b)
        mwntt.vec_axpymod(out, it["alpha"], a, q, limbs)
    torch.cuda.synchronize()
    return out


def _oracle_sample(it, ks):
    q = it["q"]
    a, b = W.to_ints(it["A"]), W.to_ints(it["B"])
    op = it["op"]
    if op == mwntt.MW_REQ_NTT_FORWARD:
        return oracle.ntt.forward_at(a, q, ks)
    if op == mwntt.MW_REQ_NTT_INVERSE:
        return oracle.ntt.inverse_at(a, q, ks)
    if op == mwntt.MW_REQ_POLYMUL:
        return oracle.polymul.negacyclic_at(a, b, q, ks)
    if op == mwntt.MW_REQ_VEC_MULMOD:
        return [a[k] * b[k] % q for k in ks]
    if op == mwntt.MW_REQ_VEC_ADDMOD:
        return [(a[k] + b[k]) % q for k in ks]
    if op == mwntt.MW_REQ_VEC_SUBMOD:
        return [(a[k] - b[k]) % q for k in ks]
    return [(it["alpha"] * a[k] + b[k]) % q for k in ks]


@pytest.mark.parametrize("budget,inflight,batch,wide,spin", [(1 << 30, 1, 32, False, 0), (1 << 30, 4, 32, False, 0),
                                                             (3 << 20, 2, 4, False, 0), (1 << 30, 3, 16, True, 0),
                                                             (1 << 30, 2, 8, False, 500)])
def test_mixed_stream_matches_alone(budget, inflight, batch, wide, spin):
    """wide: 60-, 124- and 252-bit requests in one stream; spin: the scheduler
    polls without sleeping for that many microseconds after each action."""
    require_gpu()
    import torch
    items, plans = _workload(56, seed=budget % 1000 + inflight, wide=wide)
    srv = mwntt.MwServer(budget, max_inflight=inflight, max_batch=batch, spin_us=spin)
    announce("serve mixed", budget, inflight, batch, spin)
    tickets = [srv.submit(_request(it)) for it in items]    # a burst: requests queue and batch
    outs = []
    for t, it in zip(tickets, items):
        ptr, lat = srv.result(t, wait=True)
        assert lat > 0
        outs.append(mwntt.copy_to_tensor(ptr, it["a"]))
        torch.cuda.synchronize()
        srv.release(t)
    st = srv.stats()
    assert st["completed"] == len(items) and st["pool_peak"] <= budget
    if inflight == 1:
        # requests arriving while the one stream is busy join the next batch
        assert st["max_batch_seen"] > 1
    if budget < (4 << 20):
        assert st["queue_peak"] > 1        # the small budget made requests wait
    for i, (it, out) in enumerate(zip(items, outs)):
        assert torch.equal(out, _alone(it)), f"request {i} op {it['op']}"
        if i % 5 == 0:
            ks = [0, it["n"] - 1, (i * 37) % it["n"]]
            got = host_ints(out, it["limbs"])
            assert [got[k] for k in ks] == _oracle_sample(it, ks), f"request {i}"
    srv.destroy()
    for p in plans.values():
        p.destroy()


def test_replay_poisson_gpu():
    require_gpu()
    import numpy as np
    items, plans = _workload(400, seed=9, log2_range=(10, 14))
    g = np.random.Generator(np.random.PCG64(4))
    gaps = g.exponential(1e6 / 20000.0, size=len(items))
    arrivals = list(np.cumsum(gaps) - gaps[0])
    srv = mwntt.MwServer(1 << 30, max_inflight=4, max_batch=64)
    announce("serve replay", len(items))
    lat, span = srv.replay([_request(it) for it in items], arrivals)
    assert len(lat) == len(items) and min(lat) > 0
    assert srv.stats()["completed"] == len(items)
    srv.destroy()
    for p in plans.values():
        p.destroy()


def test_one_request_at_a_time_matches_alone():
    """Each request submitted only after the previous one completed, so every
    batch holds one job (its descriptor then travels in the kernel
    arguments): transforms and products of every width at N = 2^6 .. 2^17,
    each result against the same operation alone and sampled against the
    oracle."""
    require_gpu()
    import torch
    items, plans = _workload(42, seed=31, log2_range=(6, 17), wide=True)
    srv = mwntt.MwServer(1 << 30, max_inflight=2, max_batch=8)
    announce("serve one at a time", len(items))
    for i, it in enumerate(items):
        t = srv.submit(_request(it))
        ptr, lat = srv.result(t, wait=True)
        out = mwntt.copy_to_tensor(ptr, it["a"])
        torch.cuda.synchronize()
        srv.release(t)
        assert torch.equal(out, _alone(it)), f"request {i} op {it['op']} n {it['n']} limbs {it['limbs']}"
        if i % 6 == 0:
            ks = [0, it["n"] - 1, (i * 41) % it["n"]]
            got = host_ints(out, it["limbs"])
            assert [got[k] for k in ks] == _oracle_sample(it, ks), f"request {i}"
    st = srv.stats()
    assert st["completed"] == len(items) and st["max_batch_seen"] == 1
    srv.destroy()
    for p in plans.values():
        p.destroy()


def test_mixed_stream_odd_widths():
    """A batched stream at widths inside each class (33, 80, 97, 200 and 251
    bits: Barrett on the scaled modulus in products and vec_mulmod): every
    result equals the same operation alone, and samples equal the oracle."""
    require_gpu()
    import torch
    items, plans = _workload(35, seed=47, log2_range=(6, 11), widths=[33, 80, 97, 200, 251])
    srv = mwntt.MwServer(1 << 30, max_inflight=3, max_batch=16)
    announce("serve odd widths", len(items))
    tickets = [srv.submit(_request(it)) for it in items]
    for i, (t, it) in enumerate(zip(tickets, items)):
        ptr, _ = srv.result(t, wait=True)
        out = mwntt.copy_to_tensor(ptr, it["a"])
        torch.cuda.synchronize()
        srv.release(t)
        assert torch.equal(out, _alone(it)), f"request {i} op {it['op']} bits {it['q'].bit_length()}"
        ks = [0, it["n"] - 1, (i * 37) % it["n"]]
        got = host_ints(out, it["limbs"])
        assert [got[k] for k in ks] == _oracle_sample(it, ks), f"request {i}"
    srv.destroy()
    for p in plans.values():
        p.destroy()
