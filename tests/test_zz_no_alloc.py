"""The allocation-free transform (ntt_transform_noalloc, static device
scratch) against ntt_forward / ntt_inverse through the C ABI, bit for bit:
two calls in a row per width, the second with a smaller input (the array
keeps the first call's contents), single-workgroup and two-pass sizes, and
the size limit."""
import pytest

import oracle
from paper_2509_12494_amd import mwntt
from paper_2509_12494_amd import workloads as W

from .gpu_util import announce, dev, host_ints, prime, require_gpu

pytestmark = pytest.mark.gpu

# (bits, seed, log2n, first batch, second batch): the first call of each
# two-pass case takes the large-batch configuration, the second the
# single-transform one
CASES = [(124, 2001, 16, 16, 1), (124, 2001, 17, 8, 3), (60, 11, 16, 64, 5), (252, 15, 17, 8, 2),
         (252, 15, 16, 12, 1), (124, 22, 10, 6, 2), (60, 21, 12, 9, 1)]


@pytest.mark.parametrize("bits,seed,log2n,b1,b2", CASES)
def test_noalloc_matches_plain(bits, seed, log2n, b1, b2):
    require_gpu()
    import torch
    q = prime(bits, seed)
    limbs = W.limbs_for_bits(bits)
    plan = mwntt.ntt_plan(log2n, q, limbs)
    n = plan.n
    for call, batch in enumerate((b1, b2)):
        A = W.uniform_residues(W.rng(600 + 10 * call + log2n), q, batch * n, limbs)
        a = dev(A)
        want_f, got_f = torch.empty_like(a), torch.full_like(a, -1)
        announce("noalloc forward", bits, log2n, batch, call)
        plan.forward(want_f, a, batch=batch)
        plan.transform_noalloc(False, got_f, a, batch=batch)
        torch.cuda.synchronize()
        assert torch.equal(got_f, want_f), f"forward call {call} batch {batch}"
        want_i, got_i = torch.empty_like(a), torch.full_like(a, -1)
        announce("noalloc inverse", bits, log2n, batch, call)
        plan.inverse(want_i, want_f, batch=batch)
        plan.transform_noalloc(True, got_i, want_f, batch=batch)
        torch.cuda.synchronize()
        assert torch.equal(got_i, want_i), f"inverse call {call} batch {batch}"
        assert torch.equal(got_i, a)
        ks = [0, 1, n // 2 + 3, n - 1]
        last = W.to_ints(A)[(batch - 1) * n:]
        got = host_ints(got_f, limbs)[(batch - 1) * n:]
        assert [got[k] for k in ks] == oracle.ntt.forward_at(last, q, ks)
    plan.destroy()


def test_noalloc_in_place_and_limits():
    require_gpu()
    import torch
    q = prime(252, 15)
    plan = mwntt.ntt_plan(17, q, 4)
    n = plan.n
    A = W.uniform_residues(W.rng(650), q, 2 * n, 4)
    a = dev(A)
    want = torch.empty_like(a)
    plan.forward(want, a, batch=2)
    announce("noalloc in place")
    plan.transform_noalloc(False, a, a, batch=2)          # d_out == d_in
    torch.cuda.synchronize()
    assert torch.equal(a, want)
    # 17 four-word transforms of 2^17 points need 68 MiB: above the 64 MiB array
    big = torch.empty(17 * n, 4, dtype=torch.int64, device="cuda")
    with pytest.raises(mwntt.MwError) as e:
        plan.transform_noalloc(False, big, big, batch=17)
    assert e.value.status == -3
    # direction other than 0 / 1: rejected before any device work
    assert mwntt.lib().ntt_transform_noalloc(plan._h, 2, a.data_ptr(), a.data_ptr(), 1, None) == -1
    plan.destroy()
