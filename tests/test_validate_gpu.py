"""Validate mode on the GPU: a residue >= q in any input of a BLAS call, a
plain transform, a batched run or a served request is reported as
MW_ENONCANON by mw_check or by the next entry point (which then enqueues
nothing); canonical inputs report nothing, and results with validation on
equal those with it off."""
import pytest

from paper_2509_12494_amd import mwntt
from paper_2509_12494_amd import workloads as W

from .gpu_util import announce, dev, prime, require_gpu

pytestmark = pytest.mark.gpu

WIDTHS = [(60, 11), (124, 12), (252, 15), (80, 13)]


@pytest.fixture
def validating():
    require_gpu()
    mwntt.set_validate(True)
    try:
        yield
    finally:
        mwntt.set_validate(False)
        try:
            mwntt.check()
        except mwntt.MwError:
            pass


def _inputs(q, limbs, n, seed, bad_at=None, bad_value=None):
    A = W.uniform_residues(W.rng(seed), q, n, limbs)
    if bad_at is not None:
        A[bad_at] = W.from_ints([bad_value], limbs)[0]
    return A


def _expect_noncanon(fn):
    with pytest.raises(mwntt.MwError) as e:
        fn()
    assert e.value.status == mwntt.MW_ENONCANON


@pytest.mark.parametrize("bits,seed", WIDTHS)
def test_blas_reports_noncanonical(bits, seed, validating):
    import torch
    q = prime(bits, seed)
    limbs = W.limbs_for_bits(bits)
    n = 5000
    good_a, good_b = dev(_inputs(q, limbs, n, 1)), dev(_inputs(q, limbs, n, 2))
    top = (1 << (64 * limbs)) - 1
    for op in ("vec_addmod", "vec_submod", "vec_mulmod"):
        announce("validate", op, bits)
        c = torch.empty_like(good_a)
        getattr(mwntt, op)(c, good_a, good_b, q, limbs)
        mwntt.check()                                    # canonical: nothing to report
        for which, bad_value, at in (("a", q, 0), ("b", top, n - 1)):
            bad = dev(_inputs(q, limbs, n, 3 if which == "a" else 4, at, bad_value))
            args = (bad, good_b) if which == "a" else (good_a, bad)
            getattr(mwntt, op)(c, *args, q, limbs)        # enqueued; the check runs first
            _expect_noncanon(mwntt.check)
            mwntt.check()                                 # reported once, then clear
    # the next call reports a violation found earlier and enqueues nothing
    bad = dev(_inputs(q, limbs, n, 5, 17, q + 1))
    y = good_b.clone()
    mwntt.vec_axpymod(y, 3 % q, bad, q, limbs)
    torch.cuda.synchronize()
    before = y.clone()
    _expect_noncanon(lambda: mwntt.vec_addmod(y, good_a, good_b, q, limbs))
    torch.cuda.synchronize()
    assert torch.equal(y, before)
    mwntt.vec_addmod(y, good_a, good_b, q, limbs)
    mwntt.check()


@pytest.mark.parametrize("bits,seed", [(60, 21), (124, 22), (252, 23)])
@pytest.mark.parametrize("log2n", [10, 16])
def test_transforms_report_noncanonical(log2n, bits, seed, validating):
    import torch
    q = prime(bits, seed)
    limbs = W.limbs_for_bits(bits)
    plan = mwntt.ntt_plan(log2n, q, limbs)
    n = plan.n
    good = dev(_inputs(q, limbs, 2 * n, 7))
    out = torch.empty_like(good)
    announce("validate ntt", log2n, bits)
    plan.forward(out, good, batch=2)
    plan.inverse(out, out, batch=2)
    mwntt.check()
    assert torch.equal(out, good)                        # validation does not change results
    bad = dev(_inputs(q, limbs, 2 * n, 8, 2 * n - 1, q))
    plan.forward(out, bad, batch=2)
    _expect_noncanon(mwntt.check)
    plan.inverse(out, bad, batch=2)
    _expect_noncanon(mwntt.check)
    if plan.split:
        plan.forward_pass(1, out, bad, batch=2)
        _expect_noncanon(mwntt.check)
    mwntt.check()
    plan.destroy()


def test_batch_and_server_report_noncanonical(validating):
    import torch
    q = prime(124, 42)
    plan = mwntt.ntt_plan(10, q, 2)
    n = plan.n
    a, b = dev(_inputs(q, 2, n, 9)), dev(_inputs(q, 2, n, 10))
    bad = dev(_inputs(q, 2, n, 11, 5, q))
    out = torch.empty_like(a)
    announce("validate batch")
    good_batch = mwntt.NttBatch([(plan, mwntt.NTT_JOB_POLYMUL, a, b, out)])
    good_batch.run()
    mwntt.check()
    bad_batch = mwntt.NttBatch([(plan, mwntt.NTT_JOB_POLYMUL, a, bad, out),
                                (plan, mwntt.NTT_JOB_FORWARD, a, None, torch.empty_like(a))])
    bad_batch.run()
    _expect_noncanon(mwntt.check)
    announce("validate server")
    srv = mwntt.MwServer(1 << 28, max_inflight=2, max_batch=4)
    t1 = srv.submit(mwntt.make_request(mwntt.MW_REQ_VEC_MULMOD, a, b, q=q, limbs=2, n=n))
    srv.drain()
    mwntt.check()
    t2 = srv.submit(mwntt.make_request(mwntt.MW_REQ_VEC_ADDMOD, a, bad, q=q, limbs=2, n=n))
    t3 = srv.submit(mwntt.make_request(mwntt.MW_REQ_NTT_FORWARD, bad, None, plan=plan))
    srv.drain()
    _expect_noncanon(mwntt.check)
    for t in (t1, t2, t3):
        srv.result(t, wait=True)
        srv.release(t)
    srv.destroy()
    good_batch.destroy()
    bad_batch.destroy()
    plan.destroy()
