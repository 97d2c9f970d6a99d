"""Serving scheduler on the CPU (dry-run mode: no device memory or work).

Admission never exceeds the HBM budget, admission is first-in first-out,
requests that can never fit are rejected, a tiny budget forces queueing yet
every request completes, bursts are batched, and replay records a latency for
every request.  BLAS requests are used because they need no device plan;
buffers are dummy addresses that dry-run mode never touches."""
import pytest

from paper_2509_12494_amd import mwntt
from paper_2509_12494_amd import workloads as W

Q60 = W.find_prime(60, 1)
DUMMY = 1 << 20


def _req(n, op=mwntt.MW_REQ_VEC_MULMOD):
    return mwntt.make_request(op, DUMMY, DUMMY, q=Q60, limbs=1, n=n)


def test_budget_never_exceeded_and_all_complete():
    budget = 64 * 1024
    srv = mwntt.MwServer(budget, max_inflight=2, max_batch=4, dry_run=True)
    sizes = [1000, 3000, 5000, 7000, 2000, 8000, 100, 4096] * 6
    tickets = [srv.submit(_req(n)) for n in sizes]
    for t in tickets:
        _, lat = srv.result(t, wait=True)
        assert lat >= 0
        srv.release(t)
    st = srv.stats()
    assert st["completed"] == len(sizes) and st["submitted"] == len(sizes)
    assert st["pool_peak"] <= budget
    assert st["queue_peak"] > 1              # the small budget made requests wait
    srv.destroy()


def test_fifo_admission_order():
    # one stream, one request per batch, each modelled at ~200 us so a queue
    # forms: completions follow submission order, so latencies grow
    srv = mwntt.MwServer(1 << 30, max_inflight=1, max_batch=1, dry_run=True)
    tickets = [srv.submit(_req(1_000_000 + 100 * i)) for i in range(20)]
    lats = []
    for t in tickets:
        _, lat = srv.result(t, wait=True)
        lats.append(lat)
    # request i waited for requests 0..i-1: latencies grow along the queue
    assert all(b >= a for a, b in zip(lats, lats[1:]))
    for t in tickets:
        srv.release(t)
    srv.destroy()


def test_batches_form_from_bursts():
    srv = mwntt.MwServer(1 << 26, max_inflight=1, max_batch=16, dry_run=True)
    tickets = [srv.submit(_req(1024)) for _ in range(64)]
    srv.drain()
    st = srv.stats()
    assert st["max_batch_seen"] > 1 and st["batches"] < 64
    for t in tickets:
        srv.release(t)
    srv.destroy()


def test_reject_too_large_and_invalid():
    srv = mwntt.MwServer(4096, max_inflight=1, max_batch=2, dry_run=True)
    with pytest.raises(mwntt.MwError) as e:
        srv.submit(_req(10_000))                       # 80 KB output > 4 KB budget
    assert e.value.status == -4
    with pytest.raises(mwntt.MwError) as e:
        srv.submit(mwntt.make_request(mwntt.MW_REQ_VEC_MULMOD, DUMMY, None, q=Q60, limbs=1, n=8))
    assert e.value.status == -1
    with pytest.raises(mwntt.MwError) as e:
        srv.submit(mwntt.make_request(mwntt.MW_REQ_VEC_AXPYMOD, DUMMY, DUMMY, q=Q60, limbs=1, n=8, alpha=Q60 + 1 - 1))
    assert e.value.status == -1                        # alpha not reduced
    with pytest.raises(mwntt.MwError) as e:
        srv.submit(mwntt.make_request(mwntt.MW_REQ_NTT_FORWARD, DUMMY))   # no plan
    assert e.value.status == -1
    with pytest.raises(mwntt.MwError) as e:             # n beyond the BLAS length limit
        srv.submit(mwntt.make_request(mwntt.MW_REQ_VEC_ADDMOD, DUMMY, DUMMY, q=Q60, limbs=1, n=1 << 62))
    assert e.value.status == -1
    r = mwntt.make_request(mwntt.MW_REQ_VEC_ADDMOD, DUMMY, DUMMY, q=Q60, limbs=1, n=8)
    r.limbs = 3                                         # limb counts are 1, 2 or 4
    with pytest.raises(mwntt.MwError) as e:
        srv.submit(r)
    assert e.value.status == -1
    q252 = W.find_prime(252, 6001)
    with pytest.raises(mwntt.MwError) as e:             # four-word alpha not reduced
        srv.submit(mwntt.make_request(mwntt.MW_REQ_VEC_AXPYMOD, DUMMY, DUMMY, q=q252, limbs=4, n=8, alpha=q252))
    assert e.value.status == -1
    t4 = srv.submit(mwntt.make_request(mwntt.MW_REQ_VEC_MULMOD, DUMMY, DUMMY, q=q252, limbs=4, n=8))
    srv.result(t4, wait=True)
    srv.release(t4)
    t = srv.submit(_req(100))
    assert srv.result(t, wait=True)[0] is None          # dry run: no output buffer
    with pytest.raises(mwntt.MwError):
        srv.result(t + 1000, wait=False)                # unknown ticket
    srv.release(t)
    srv.destroy()


def test_replay_poisson_stream():
    import numpy as np
    g = np.random.Generator(np.random.PCG64(3))
    count = 2000
    gaps = g.exponential(1e6 / 20000.0, size=count)     # 20k requests/s
    arrivals = list(np.cumsum(gaps) - gaps[0])
    sizes = np.floor(2.0 ** g.uniform(10, 14, size=count)).astype(int)
    reqs = [_req(int(n)) for n in sizes]
    srv = mwntt.MwServer(1 << 24, max_inflight=4, max_batch=32, dry_run=True)
    lat, span = srv.replay(reqs, arrivals)
    assert len(lat) == count and min(lat) >= 0
    assert span >= arrivals[-1]
    st = srv.stats()
    assert st["completed"] == count
    srv.destroy()


def test_config_errors():
    with pytest.raises(mwntt.MwError):
        mwntt.MwServer(1 << 20, max_inflight=0, dry_run=True)
    with pytest.raises(mwntt.MwError):
        mwntt.MwServer(1 << 20, max_batch=1000, dry_run=True)
    with pytest.raises(mwntt.MwError):
        mwntt.MwServer(1 << 20, spin_us=200000, dry_run=True)
    with pytest.raises(mwntt.MwError):
        mwntt.MwServer(1 << 20, resident=True, resident_max_tiles=4097, dry_run=True)


def test_spinning_scheduler_completes_stream():
    # a scheduler that polls without sleeping between actions serves the same
    # requests as a sleeping one
    reqs = [_req(1024 + 37 * i) for i in range(300)]
    arrivals = [20.0 * i for i in range(300)]
    srv = mwntt.MwServer(1 << 24, max_inflight=2, max_batch=8, dry_run=True, spin_us=500)
    lat, span = srv.replay(reqs, arrivals)
    assert len(lat) == 300 and min(lat) >= 0 and span >= arrivals[-1]
    assert srv.stats()["completed"] == 300
    srv.destroy()


def test_resident_flag_ignored_in_dry_run():
    # the device-resident loop needs a device: a dry run keeps the slot path
    srv = mwntt.MwServer(1 << 24, max_inflight=2, max_batch=8, dry_run=True, resident=True)
    tickets = [srv.submit(_req(1024 + i)) for i in range(20)]
    for t in tickets:
        srv.result(t, wait=True)
        srv.release(t)
    st = srv.stats()
    assert st["completed"] == 20 and st["resident_requests"] == 0 and st["resident_launches"] == 0
    srv.destroy()
