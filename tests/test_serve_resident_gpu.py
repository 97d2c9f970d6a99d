"""The serving runtime's device-resident request loop on the GPU: one
persistent kernel takes one- and two-word transform, product and BLAS requests
of up to resident_max_tiles tiles from a ring in mapped host memory; the
others keep the slot path.  Every result equals the same operation run alone
through the plain entry points (and the oracle on sampled outputs): in a
burst with the default routing and with every request in the loop, one
request at a time (N = 2^6 .. 2^17, widths inside each class), mixed with
four-word requests that keep the slot path, at the largest product (2^17,
124-bit) and after the loop has left on idling and been launched again, and
with inputs rewritten and plans replaced between requests.  The routing
follows the tile counts."""
import time

import pytest

from paper_2509_12494_amd import mwntt

from .gpu_util import announce, host_ints, require_gpu
from .test_serve_gpu import _alone, _oracle_sample, _request, _workload

pytestmark = pytest.mark.gpu

BLAS_TILE = 1024       # residues per BLAS tile of the loop
DEFAULT_TILES = 4096   # the default routing bound: every request the loop can take


def _tiles(it):
    """Workgroup tiles of a request (a transform's or product's are the batched
    executor's)."""
    import torch
    if it["plan"] is None:
        return -(-it["n"] // BLAS_TILE)
    op = {mwntt.MW_REQ_NTT_FORWARD: mwntt.NTT_JOB_FORWARD, mwntt.MW_REQ_NTT_INVERSE: mwntt.NTT_JOB_INVERSE,
          mwntt.MW_REQ_POLYMUL: mwntt.NTT_JOB_POLYMUL}[it["op"]]
    out = torch.empty_like(it["a"])
    b = mwntt.NttBatch([(it["plan"], op, it["a"], it["b"] if op == mwntt.NTT_JOB_POLYMUL else None, out)])
    t = b.info()["tiles"]
    b.destroy()
    return t


def _in_loop(items, max_tiles):
    bound = max_tiles or DEFAULT_TILES
    return sum(1 for it in items if it["limbs"] <= 2 and _tiles(it) <= bound)


def _run_and_check(srv, items, serial, sample_every=3):
    import torch
    tickets = [] if serial else [srv.submit(_request(it)) for it in items]
    for i, it in enumerate(items):
        t = srv.submit(_request(it)) if serial else tickets[i]
        ptr, lat = srv.result(t, wait=True)
        assert lat > 0
        out = mwntt.copy_to_tensor(ptr, it["a"])
        torch.cuda.synchronize()
        srv.release(t)
        assert torch.equal(out, _alone(it)), \
            f"request {i} op {it['op']} n {it['n']} bits {it['q'].bit_length()}"
        if i % sample_every == 0:
            ks = [0, it["n"] - 1, (i * 37) % it["n"]]
            got = host_ints(out, it["limbs"])
            assert [got[k] for k in ks] == _oracle_sample(it, ks), f"request {i}"


@pytest.mark.parametrize("wide,max_tiles", [(False, 0), (True, 0), (False, 16), (True, 16)])
def test_resident_burst_matches_alone(wide, max_tiles):
    """A burst of 56 requests (wide: a third of them 252-bit, which take the
    slot path beside the loop; max_tiles 16: requests of more tiles take the
    slot path too)."""
    require_gpu()
    items, plans = _workload(56, seed=71 + wide, wide=wide, log2_range=(10, 15))
    srv = mwntt.MwServer(1 << 30, max_inflight=3, max_batch=16, resident=True, resident_max_tiles=max_tiles)
    announce("resident burst", wide, max_tiles)
    _run_and_check(srv, items, serial=False)
    st = srv.stats()
    assert st["completed"] == len(items)
    expect = _in_loop(items, max_tiles)
    assert st["resident_requests"] == expect and st["resident_launches"] >= 1
    if max_tiles or wide:
        assert 0 < expect < len(items)      # both paths in use
    srv.destroy()
    for p in plans.values():
        p.destroy()


def test_resident_one_at_a_time():
    """Each request submitted after the previous one completed: transforms
    and products at N = 2^6 .. 2^17 and BLAS at ragged lengths, at 33, 60,
    80, 97 and 124 bits (Barrett on the scaled modulus below the top of a
    class)."""
    require_gpu()
    items, plans = _workload(45, seed=83, log2_range=(6, 17), widths=[33, 60, 80, 97, 124])
    srv = mwntt.MwServer(1 << 30, max_inflight=2, max_batch=8, resident=True, resident_max_tiles=4096)
    announce("resident one at a time", len(items))
    _run_and_check(srv, items, serial=True)
    assert srv.stats()["resident_requests"] == len(items)
    srv.destroy()
    for p in plans.values():
        p.destroy()


def test_resident_largest_job():
    """A 124-bit negacyclic product at N = 2^17 (the largest plan): 512 tiles
    in three phases."""
    require_gpu()
    import torch
    from paper_2509_12494_amd import workloads as W
    q = W.find_prime(124, 97)
    g = W.rng(97)
    n = 1 << 17
    A, B = W.uniform_residues(g, q, n, 2), W.uniform_residues(g, q, n, 2)
    plan = mwntt.ntt_plan(17, q, 2)
    it = dict(op=mwntt.MW_REQ_POLYMUL, q=q, limbs=2, n=n, plan=plan, A=A, B=B,
              a=mwntt.to_device(A), b=mwntt.to_device(B), alpha=0)
    srv = mwntt.MwServer(1 << 30, max_inflight=2, max_batch=8, resident=True, resident_max_tiles=4096)
    announce("resident 2^17 product")
    _run_and_check(srv, [it], serial=True, sample_every=1)
    assert srv.stats()["resident_requests"] == 1
    srv.destroy()
    plan.destroy()
    torch.cuda.synchronize()


def test_resident_relaunch_after_idle():
    """The loop leaves after 20 ms without work; the next request launches
    it again, and results stay exact."""
    require_gpu()
    items, plans = _workload(21, seed=89, log2_range=(8, 12))
    srv = mwntt.MwServer(1 << 30, max_inflight=2, max_batch=8, resident=True)
    announce("resident relaunch")
    for part in (items[:7], items[7:14], items[14:]):
        _run_and_check(srv, part, serial=False)
        time.sleep(0.1)
    st = srv.stats()
    assert st["resident_requests"] == len(items)
    assert st["resident_launches"] >= 3
    srv.destroy()
    for p in plans.values():
        p.destroy()


def test_resident_replay_poisson():
    """An open-loop Poisson replay at 20 K requests/s completes every request
    through the loop."""
    require_gpu()
    import numpy as np
    items, plans = _workload(400, seed=9, log2_range=(10, 14))
    g = np.random.Generator(np.random.PCG64(4))
    gaps = g.exponential(1e6 / 20000.0, size=len(items))
    arrivals = list(np.cumsum(gaps) - gaps[0])
    srv = mwntt.MwServer(1 << 30, max_inflight=4, max_batch=64, resident=True)
    announce("resident replay", len(items))
    lat, span = srv.replay([_request(it) for it in items], arrivals)
    assert len(lat) == len(items) and min(lat) > 0
    st = srv.stats()
    assert st["completed"] == len(items) and st["resident_requests"] == _in_loop(items, 0)
    srv.destroy()
    for p in plans.values():
        p.destroy()


def test_resident_slot_path_not_held_behind_the_loop():
    """Requests routed to the slot path (more than 16 tiles) in an open-loop
    replay of 4000 requests: a slot batch whose stream shares the loop's
    hardware queue makes the loop yield after 0.5 ms, so no request waits
    for the replay to end (before the yield, one waited the whole replay)."""
    require_gpu()
    import numpy as np
    items, plans = _workload(4000, seed=17, log2_range=(10, 15))
    g = np.random.Generator(np.random.PCG64(6))
    gaps = g.exponential(1e6 / 20000.0, size=len(items))
    arrivals = list(np.cumsum(gaps) - gaps[0])
    srv = mwntt.MwServer(1 << 30, max_inflight=4, max_batch=64, resident=True, resident_max_tiles=16)
    announce("resident yield", len(items))
    lat, span = srv.replay([_request(it) for it in items], arrivals)
    st = srv.stats()
    assert st["completed"] == len(items) and 0 < st["resident_requests"] < len(items)
    assert max(lat) < 100e3, (max(lat), st["resident_yields"])
    srv.destroy()
    for p in plans.values():
        p.destroy()


def test_resident_dependency_wait_bound_fails_requests_cleanly():
    """A tile's wait for the earlier phases of its request bounded at 1 us
    (forced from the host): tiles of two-phase 2^16 transforms give up, their
    requests complete as failed (MW_EDEVICE) instead of hanging, every request
    that did not fail is exact, the loop ends normally, and a server with the
    default bound afterwards is exact again."""
    require_gpu()
    import torch
    items, plans = _workload(12, seed=103, log2_range=(16, 16), widths=[124])
    items = [it for it in items if it["plan"] is not None]
    srv = mwntt.MwServer(1 << 30, max_inflight=2, max_batch=8, resident=True, resident_wait_us=1)
    announce("resident wait bound", len(items))
    tickets = [srv.submit(_request(it)) for it in items]
    failed = 0
    for i, (t, it) in enumerate(zip(tickets, items)):
        try:
            ptr, _ = srv.result(t, wait=True)
        except mwntt.MwError as e:
            assert e.status == -5, e          # MW_EDEVICE
            failed += 1
            srv.release(t)
            continue
        out = mwntt.copy_to_tensor(ptr, it["a"])
        torch.cuda.synchronize()
        srv.release(t)
        assert torch.equal(out, _alone(it)), f"request {i}"
    assert failed >= 1
    assert srv.stats()["completed"] == len(items)
    srv.destroy()
    srv = mwntt.MwServer(1 << 30, max_inflight=2, max_batch=8, resident=True)
    _run_and_check(srv, items[:4], serial=False, sample_every=4)
    srv.destroy()
    for p in plans.values():
        p.destroy()


def test_resident_validate_mode_keeps_slot_path():
    """In validate mode every request takes the slot path (its inputs are
    checked on a slot's stream)."""
    require_gpu()
    items, plans = _workload(7, seed=101)
    prev = mwntt.get_validate()
    mwntt.set_validate(True)
    try:
        srv = mwntt.MwServer(1 << 30, max_inflight=2, max_batch=8, resident=True)
        announce("resident validate mode")
        _run_and_check(srv, items, serial=False)
        assert srv.stats()["resident_requests"] == 0
        srv.destroy()
    finally:
        mwntt.set_validate(prev)
    for p in plans.values():
        p.destroy()


def test_resident_rewritten_inputs_and_replaced_plans():
    """Device memory that changes while the loop runs: one input buffer is
    rewritten (a device copy, completed before each submit) between requests,
    and plans are destroyed and created again with other moduli, whose tables
    may land at the addresses of the old ones.  Each result follows the new
    contents: a tile reads its inputs and tables after an L2 invalidate on its
    XCD, and what earlier phases wrote with device-scope loads.  Transforms of
    2^16 (two phases, 256 tiles) and 2^12, and vec_mulmod of 2^16 residues."""
    require_gpu()
    import torch
    from paper_2509_12494_amd import workloads as W
    n = 1 << 16
    srv = mwntt.MwServer(1 << 30, max_inflight=2, max_batch=8, resident=True, resident_max_tiles=4096)
    announce("resident: rewritten inputs, replaced plans")
    for rep in range(6):
        q = W.find_prime(124, 600 + rep)
        g = W.rng(600 + rep)
        plans = {16: mwntt.ntt_plan(16, q, 2), 12: mwntt.ntt_plan(12, q, 2)}
        a = mwntt.to_device(W.uniform_residues(g, q, n, 2))
        b = mwntt.to_device(W.uniform_residues(g, q, n, 2))
        for k in range(3):
            # new contents in the same buffer for each request
            a.copy_(mwntt.to_device(W.uniform_residues(g, q, n, 2)))
            torch.cuda.synchronize()
            items = [dict(op=mwntt.MW_REQ_NTT_FORWARD, q=q, limbs=2, n=n, plan=plans[16], a=a, b=None, alpha=0),
                     dict(op=mwntt.MW_REQ_NTT_INVERSE, q=q, limbs=2, n=1 << 12, plan=plans[12],
                          a=a[:1 << 12], b=None, alpha=0),
                     dict(op=mwntt.MW_REQ_VEC_MULMOD, q=q, limbs=2, n=n, plan=None, a=a, b=b, alpha=0)]
            for it in items:
                t = srv.submit(_request(it))
                ptr, lat = srv.result(t, wait=True)
                out = mwntt.copy_to_tensor(ptr, it["a"])
                torch.cuda.synchronize()
                srv.release(t)
                assert torch.equal(out, _alone(it)), f"rep {rep} request {k} op {it['op']}"
        for p in plans.values():
            p.destroy()
    assert srv.stats()["resident_requests"] == 6 * 3 * 3
    srv.destroy()
