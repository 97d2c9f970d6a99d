"""The batched executor against the oracle, bit for bit.

Mixed lengths and modulus widths in one run (forward, inverse, fused
products), repeated runs of one batch, hipGraph capture with several replays
interleaved with eager work, and the paper-scale
mixed batch (96 polynomials, N = 2^12..2^16, 60/124-bit) and fused products
(256 pairs at N = 2^14) on sampled outputs."""
import functools

import pytest

import oracle
from paper_2509_12494_amd import mwntt
from paper_2509_12494_amd import workloads as W

from .gpu_util import announce, bitrev, dev, host_ints, prime, require_gpu

pytestmark = pytest.mark.gpu


@functools.lru_cache(maxsize=None)
def _plan(log2n, bits, seed):
    return mwntt.ntt_plan(log2n, prime(bits, seed), W.limbs_for_bits(bits))


def _jobs_small():
    """Mixed small jobs whose outputs the oracle computes in full."""
    specs = []
    for i, (log2n, bits) in enumerate([(6, 60), (6, 124), (7, 124), (8, 60), (9, 124), (10, 60), (10, 124),
                                       (7, 60), (8, 124)]):
        specs.append((log2n, bits, 40 + i % 3))
    return specs


def test_mixed_forward_inverse_product_small():
    require_gpu()
    import torch
    jobs, checks = [], []
    for k, (log2n, bits, seed) in enumerate(_jobs_small()):
        plan = _plan(log2n, bits, seed)
        q, limbs, n = plan.q, plan.limbs, plan.n
        g = W.rng(500 + k)
        A = W.uniform_residues(g, q, n, limbs)
        B = W.uniform_residues(g, q, n, limbs)
        a, b = dev(A), dev(B)
        op = k % 3
        out = torch.empty_like(a)
        a_i, b_i = W.to_ints(A), W.to_ints(B)
        if op == 0:
            jobs.append((plan, mwntt.NTT_JOB_FORWARD, a, None, out))
            checks.append((out, limbs, oracle.ntt.ntt_negacyclic(a_i, q)))
        elif op == 1:
            jobs.append((plan, mwntt.NTT_JOB_INVERSE, a, None, out))
            checks.append((out, limbs, oracle.ntt.intt_negacyclic(a_i, q)))
        else:
            jobs.append((plan, mwntt.NTT_JOB_POLYMUL, a, b, out))
            checks.append((out, limbs, oracle.polymul.negacyclic(a_i, b_i, q)))
    batch = mwntt.NttBatch(jobs)
    announce("batch small", batch.info())
    for rep in range(3):
        for out, _, _ in checks:
            out.zero_()
        batch.run()
        batch.check()
        for i, (out, limbs, want) in enumerate(checks):
            assert host_ints(out, limbs) == want, f"run {rep} job {i}"
    batch.destroy()


def test_graph_capture_replays():
    require_gpu()
    import torch
    plan60, plan124 = _plan(9, 60, 41), _plan(11, 124, 42)
    A = W.uniform_residues(W.rng(7), plan60.q, plan60.n, 1)
    B = W.uniform_residues(W.rng(8), plan124.q, plan124.n, 2)
    C = W.uniform_residues(W.rng(9), plan124.q, plan124.n, 2)
    a, b, c = dev(A), dev(B), dev(C)
    oa, ob = torch.empty_like(a), torch.empty_like(b)
    batch = mwntt.NttBatch([(plan60, mwntt.NTT_JOB_FORWARD, a, None, oa),
                            (plan124, mwntt.NTT_JOB_POLYMUL, b, c, ob)])
    want_a = oracle.ntt.ntt_negacyclic(W.to_ints(A), plan60.q)
    n = plan124.n
    ks = [0, 1, n // 2, n - 1]
    want_b = oracle.polymul.negacyclic_at(W.to_ints(B), W.to_ints(C), plan124.q, ks)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        batch.run(stream=s)
    torch.cuda.synchronize()
    for rep in range(4):
        oa.zero_()
        ob.fill_(0)
        torch.cuda.synchronize()
        announce("graph replay", rep)
        g.replay()
        torch.cuda.synchronize()
        assert host_ints(oa, 1) == want_a, rep
        got = host_ints(ob, 2)
        assert [got[k] for k in ks] == want_b, rep
        batch.run()            # eager run between replays
        batch.check()
        assert host_ints(oa, 1) == want_a, rep
    del g
    batch.destroy()


def test_paper_mixed_batch_96():
    """96 polynomials, N uniform over 2^12..2^16, even index 60-bit, odd 124-bit."""
    require_gpu()
    import torch
    polys = W.config_batched()
    jobs, plain = [], []
    plans = {}
    for i, (log2n, q, limbs, coeffs) in enumerate(polys):
        if (log2n, q) not in plans:
            plans[(log2n, q)] = mwntt.ntt_plan(log2n, q, limbs)
        plan = plans[(log2n, q)]
        x = dev(coeffs)
        y = torch.empty_like(x)
        jobs.append((plan, mwntt.NTT_JOB_FORWARD, x, None, y))
        plain.append((plan, x, y, limbs, q, log2n))
    batch = mwntt.NttBatch(jobs)
    announce("batch 96", batch.info())
    batch.run()
    batch.check()
    for i, (plan, x, y, limbs, q, log2n) in enumerate(plain):
        ref = torch.empty_like(x)
        plan.forward(ref, x)
        torch.cuda.synchronize()
        assert torch.equal(ref, y), f"job {i}"
        if i % 16 == 0:
            n = 1 << log2n
            a = host_ints(x, limbs)
            got = host_ints(y, limbs)
            ks = [0, n - 1, (i * 7919) % n]
            assert [got[k] for k in ks] == oracle.ntt.forward_at(a, q, ks), f"job {i}"
    # and back: inverse jobs restore every input
    inv_jobs = [(p, mwntt.NTT_JOB_INVERSE, y, None, y) for (p, x, y, _, _, _) in plain]
    binv = mwntt.NttBatch(inv_jobs)
    binv.run()
    binv.check()
    for i, (plan, x, y, limbs, q, log2n) in enumerate(plain):
        assert torch.equal(x, y), f"job {i}"
    batch.destroy()
    binv.destroy()


def test_paper_fused_products_256():
    """256 negacyclic products at N = 2^14, 124-bit, sampled against schoolbook."""
    require_gpu()
    import torch
    q, A, B = W.config_fused()
    pairs, n = A.shape[0], A.shape[1]
    plan = mwntt.ntt_plan(14, q, 2)
    a = dev(A.reshape(-1, 2))
    b = dev(B.reshape(-1, 2))
    c = torch.empty_like(a)
    jobs = [(plan, mwntt.NTT_JOB_POLYMUL, a[i * n:(i + 1) * n], b[i * n:(i + 1) * n], c[i * n:(i + 1) * n])
            for i in range(pairs)]
    batch = mwntt.NttBatch(jobs)
    announce("fused 256", batch.info())
    batch.run()
    batch.check()
    for i in (0, 1, 97, 255):
        ai = W.to_ints(A[i])
        bi = W.to_ints(B[i])
        got = host_ints(c[i * n:(i + 1) * n], 2)
        ks = [0, 1, n // 2, n - 1, (i * 131) % n]
        assert [got[k] for k in ks] == oracle.polymul.negacyclic_at(ai, bi, q, ks), f"pair {i}"
    # the whole product of pair 5 equals plain forward / vec_mulmod / inverse
    fa, fb = torch.empty(n, 2, dtype=torch.int64, device="cuda"), torch.empty(n, 2, dtype=torch.int64, device="cuda")
    plan.forward(fa, a[5 * n:6 * n])
    plan.forward(fb, b[5 * n:6 * n])
    mwntt.vec_mulmod(fa, fa, fb, q, 2)
    plan.inverse(fb, fa)
    torch.cuda.synchronize()
    assert torch.equal(fb, c[5 * n:6 * n])
    batch.destroy()


@pytest.mark.parametrize("bits", [60, 124])
def test_largest_length_all_ops(bits):
    """N = 2^17 (the largest length the serving stream draws): forward, inverse
    and product jobs in one batch, against the plain entry points and sampled
    oracle outputs."""
    require_gpu()
    import torch
    plan = _plan(17, bits, 43)
    q, limbs, n = plan.q, plan.limbs, plan.n
    g = W.rng(600 + bits)
    A = W.uniform_residues(g, q, n, limbs)
    B = W.uniform_residues(g, q, n, limbs)
    a, b = dev(A), dev(B)
    fo, io, mo = torch.empty_like(a), torch.empty_like(a), torch.empty_like(a)
    batch = mwntt.NttBatch([(plan, mwntt.NTT_JOB_FORWARD, a, None, fo), (plan, mwntt.NTT_JOB_INVERSE, a, None, io),
                            (plan, mwntt.NTT_JOB_POLYMUL, a, b, mo)])
    announce("batch 2^17", bits, batch.info())
    batch.run()
    batch.check()
    ref = torch.empty_like(a)
    plan.forward(ref, a)
    torch.cuda.synchronize()
    assert torch.equal(ref, fo)
    plan.inverse(ref, a)
    torch.cuda.synchronize()
    assert torch.equal(ref, io)
    a_i, b_i = W.to_ints(A), W.to_ints(B)
    ks = [0, 1, n // 2, n - 1, 77777]
    got = host_ints(fo, limbs)
    assert [got[k] for k in ks] == oracle.ntt.forward_at(a_i, q, ks)
    got = host_ints(io, limbs)
    assert [got[k] for k in ks] == oracle.ntt.inverse_at(a_i, q, ks)
    got = host_ints(mo, limbs)
    assert [got[k] for k in ks[:3]] == oracle.polymul.negacyclic_at(a_i, b_i, q, ks[:3])
    batch.destroy()


def test_three_widths_in_one_batch():
    """60-, 124- and 252-bit jobs (forward, inverse, product; N = 2^6..2^10) in
    one batch: the four-word tiles run in a kernel of their own in each phase;
    every output against the oracle in full."""
    require_gpu()
    import torch
    specs = [(6, 252), (7, 60), (8, 124), (8, 252), (9, 252), (10, 124), (10, 252), (7, 252), (9, 60)]
    jobs, checks = [], []
    for k, (log2n, bits) in enumerate(specs):
        plan = _plan(log2n, bits, 45 + k % 2)
        q, limbs, n = plan.q, plan.limbs, plan.n
        g = W.rng(800 + k)
        A, B = W.uniform_residues(g, q, n, limbs), W.uniform_residues(g, q, n, limbs)
        a, b = dev(A), dev(B)
        out = torch.empty_like(a)
        a_i, b_i = W.to_ints(A), W.to_ints(B)
        op = k % 3
        if op == 0:
            jobs.append((plan, mwntt.NTT_JOB_FORWARD, a, None, out))
            checks.append((out, limbs, oracle.ntt.ntt_negacyclic(a_i, q)))
        elif op == 1:
            jobs.append((plan, mwntt.NTT_JOB_INVERSE, a, None, out))
            checks.append((out, limbs, oracle.ntt.intt_negacyclic(a_i, q)))
        else:
            jobs.append((plan, mwntt.NTT_JOB_POLYMUL, a, b, out))
            checks.append((out, limbs, oracle.polymul.negacyclic(a_i, b_i, q)))
    batch = mwntt.NttBatch(jobs)
    info = batch.info()
    announce("batch three widths", info)
    # one launch per phase for the one- and two-word tiles (products present:
    # three phases) and one per phase for the four-word tiles (no product: two)
    assert info["launches"] == 3 + 2
    for rep in range(2):
        for out, _, _ in checks:
            out.zero_()
        batch.run()
        batch.check()
        for i, (out, limbs, want) in enumerate(checks):
            assert host_ints(out, limbs) == want, f"run {rep} job {i}"
    batch.destroy()


def test_252bit_product_2e16_sampled():
    """A 252-bit negacyclic product at N = 2^16 through the executor, against
    plain forward / vec_mulmod / inverse and sampled schoolbook outputs."""
    require_gpu()
    import torch
    plan = _plan(16, 252, 47)
    q, n = plan.q, plan.n
    g = W.rng(900)
    A, B = W.uniform_residues(g, q, n, 4), W.uniform_residues(g, q, n, 4)
    a, b = dev(A), dev(B)
    c = torch.empty_like(a)
    batch = mwntt.NttBatch([(plan, mwntt.NTT_JOB_POLYMUL, a, b, c)])
    batch.run()
    batch.check()
    fa, fb = torch.empty_like(a), torch.empty_like(b)
    plan.forward(fa, a)
    plan.forward(fb, b)
    mwntt.vec_mulmod(fa, fa, fb, q, 4)
    plan.inverse(fb, fa)
    torch.cuda.synchronize()
    assert torch.equal(fb, c)
    ks = [0, 1, n // 2, n - 1]
    got = host_ints(c, 4)
    assert [got[k] for k in ks] == oracle.polymul.negacyclic_at(W.to_ints(A), W.to_ints(B), q, ks)
    batch.destroy()


def _plain(plan, op, a, b):
    """The job through the plain entry points."""
    import torch
    out = torch.empty_like(a)
    if op == mwntt.NTT_JOB_FORWARD:
        plan.forward(out, a)
    elif op == mwntt.NTT_JOB_INVERSE:
        plan.inverse(out, a)
    else:
        fa, fb = torch.empty_like(a), torch.empty_like(b)
        plan.forward(fa, a)
        plan.forward(fb, b)
        mwntt.vec_mulmod(fa, fa, fb, plan.q, plan.limbs)
        plan.inverse(out, fa)
    return out


@pytest.mark.parametrize("seed", [1, 2])
def test_random_mixes_match_plain(seed):
    """Seeded random batches: 40 jobs, each of random width (60 / 124 / 252
    bits), N = 2^6..2^14, op and order flags; every output equal to the same
    job through the plain entry points, and sampled outputs to the oracle."""
    require_gpu()
    import torch
    g = W.rng(9100 + seed)
    jobs, refs = [], []
    for k in range(40):
        bits = int(g.choice([60, 124, 252]))
        log2n = int(g.integers(6, 15))
        op = int(g.integers(0, 3))
        flags = int(g.integers(0, 4)) if op != mwntt.NTT_JOB_POLYMUL else 0
        q = prime(bits, 50 + k % 3)
        limbs = W.limbs_for_bits(bits)
        plan = mwntt.ntt_plan(log2n, q, limbs, flags=flags)
        n = plan.n
        A, B = W.uniform_residues(g, q, n, limbs), W.uniform_residues(g, q, n, limbs)
        a, b = dev(A), dev(B)
        out = torch.empty_like(a)
        jobs.append((plan, op, a, b if op == mwntt.NTT_JOB_POLYMUL else None, out))
        refs.append((plan, op, a, b, out, A, B, flags))
    batch = mwntt.NttBatch(jobs)
    announce("random mix", seed, batch.info())
    batch.run()
    batch.check()
    for i, (plan, op, a, b, out, A, B, flags) in enumerate(refs):
        want = _plain(plan, op, a, b)
        torch.cuda.synchronize()
        assert torch.equal(out, want), f"job {i}: op {op}, N {plan.n}, {plan.limbs} limbs, flags {flags}"
        if i % 8 == 0:
            n, q = plan.n, plan.q
            ks = [0, n - 1, (i * 131) % n]
            got = host_ints(out, plan.limbs)
            a_i, b_i = W.to_ints(A), W.to_ints(B)
            if op == mwntt.NTT_JOB_POLYMUL:
                assert [got[k] for k in ks] == oracle.polymul.negacyclic_at(a_i, b_i, q, ks)
            elif op == mwntt.NTT_JOB_FORWARD:
                pos = [bitrev(k, plan.log2n) if flags & mwntt.NTT_BITREV_OUT else k for k in ks]
                assert [got[p_] for p_ in pos] == oracle.ntt.forward_at(a_i, q, ks)
            else:
                src = a_i
                if flags & mwntt.NTT_BITREV_IN:     # input is a spectrum in bit-reversed order
                    src = [a_i[bitrev(k, plan.log2n)] for k in range(n)]
                assert [got[k] for k in ks] == oracle.ntt.inverse_at(src, q, ks)
    batch.destroy()
    for plan, *_ in refs:
        plan.destroy()


@pytest.mark.parametrize("bits", [60, 124, 252])
def test_single_width_batches_match_plain(bits):
    """A batch of one modulus width runs that width's kernel, whose tiles of
    2^5 .. 2^9-point lines have compile-time code: forward (natural and
    bit-reversed output), inverse (natural and bit-reversed input) and
    products for N = 2^8 .. 2^17, every output equal to the plain entry
    points, sampled outputs to the oracle."""
    require_gpu()
    import torch
    limbs = W.limbs_for_bits(bits)
    g = W.rng(9300 + bits)
    jobs, refs = [], []
    for log2n in range(8, 18):
        for op in (mwntt.NTT_JOB_FORWARD, mwntt.NTT_JOB_INVERSE, mwntt.NTT_JOB_POLYMUL):
            if op == mwntt.NTT_JOB_POLYMUL and bits == 252 and log2n > 15:
                continue   # keeps the four-word case within the test's time
            flags = 0
            if op == mwntt.NTT_JOB_FORWARD and log2n % 2:
                flags = mwntt.NTT_BITREV_OUT
            if op == mwntt.NTT_JOB_INVERSE and log2n % 2 == 0:
                flags = mwntt.NTT_BITREV_IN
            q = prime(bits, 60 + log2n % 2)
            plan = mwntt.ntt_plan(log2n, q, limbs, flags=flags)
            n = plan.n
            A, B = W.uniform_residues(g, q, n, limbs), W.uniform_residues(g, q, n, limbs)
            a, b = dev(A), dev(B)
            out = torch.empty_like(a)
            jobs.append((plan, op, a, b if op == mwntt.NTT_JOB_POLYMUL else None, out))
            refs.append((plan, op, a, b, out, A, B, flags))
    batch = mwntt.NttBatch(jobs)
    info = batch.info()
    announce("single width", bits, info)
    assert info["launches"] == 3          # one width: one launch per phase
    batch.run()
    batch.check()
    for i, (plan, op, a, b, out, A, B, flags) in enumerate(refs):
        want = _plain(plan, op, a, b)
        torch.cuda.synchronize()
        assert torch.equal(out, want), f"job {i}: op {op}, N {plan.n}, flags {flags}"
        if i % 4 == 0:
            n, q = plan.n, plan.q
            ks = [0, n - 1, (i * 977) % n]
            got = host_ints(out, plan.limbs)
            a_i, b_i = W.to_ints(A), W.to_ints(B)
            if op == mwntt.NTT_JOB_POLYMUL:
                assert [got[k] for k in ks] == oracle.polymul.negacyclic_at(a_i, b_i, q, ks)
            elif op == mwntt.NTT_JOB_FORWARD:
                pos = [bitrev(k, plan.log2n) if flags & mwntt.NTT_BITREV_OUT else k for k in ks]
                assert [got[p_] for p_ in pos] == oracle.ntt.forward_at(a_i, q, ks)
            else:
                src = a_i
                if flags & mwntt.NTT_BITREV_IN:
                    src = [a_i[bitrev(k, plan.log2n)] for k in range(n)]
                assert [got[k] for k in ks] == oracle.ntt.inverse_at(src, q, ks)
    batch.destroy()
    for plan, *_ in refs:
        plan.destroy()


def test_rns_products_recombine_by_crt():
    """One product of polynomials mod Q = q_1*...*q_4 (two 124-bit and two
    60-bit primes, N = 2^12) held in RNS form: four product jobs, one per
    prime, in one batch; the Chinese-remainder recombination of the four
    results equals the product mod Q (sampled, from the definition)."""
    require_gpu()
    import torch
    widths = [(124, 71), (124, 72), (60, 73), (60, 74)]
    Q = 1
    for bits, seed in widths:
        Q *= prime(bits, seed)
    log2n, n = 12, 1 << 12
    g = W.rng(7100)
    a = W.uniform_ints(g, Q, n)
    b = W.uniform_ints(g, Q, n)
    jobs, outs = [], []
    for bits, seed in widths:
        q, limbs = prime(bits, seed), W.limbs_for_bits(bits)
        plan = _plan(log2n, bits, seed)
        x = dev(W.from_ints([v % q for v in a], limbs))
        y = dev(W.from_ints([v % q for v in b], limbs))
        c = torch.empty_like(x)
        jobs.append((plan, mwntt.NTT_JOB_POLYMUL, x, y, c))
        outs.append((q, limbs, c))
    batch = mwntt.NttBatch(jobs)
    announce("rns product", batch.info())
    batch.run()
    batch.check()
    ks = [0, 1, n // 3, n - 1]
    res = [0] * len(ks)
    for q, limbs, c in outs:
        got = host_ints(c, limbs)
        m = Q // q
        coef = m * pow(m, -1, q)
        for i, k in enumerate(ks):
            res[i] = (res[i] + got[k] * coef) % Q
    assert res == oracle.polymul.negacyclic_at(a, b, Q, ks)
    batch.destroy()


def test_batch_argument_errors():
    require_gpu()
    import torch
    plan = _plan(5, 124, 42)          # N = 2^5: below the executor's 2^6
    x = torch.zeros(32, 2, dtype=torch.int64, device="cuda")
    with pytest.raises(mwntt.MwError) as e:
        mwntt.NttBatch([(plan, mwntt.NTT_JOB_FORWARD, x, None, x)])
    assert e.value.status == -3
    p60 = mwntt.ntt_plan(8, (1 << 31) * 0 + prime(60, 41), 1)
    y = torch.zeros(256, 1, dtype=torch.int64, device="cuda")
    with pytest.raises(mwntt.MwError):
        mwntt.NttBatch([(p60, mwntt.NTT_JOB_POLYMUL, y, None, y)])   # product without b
    p60.destroy()


@pytest.mark.parametrize("bits", [60, 124, 252])
def test_single_job_batches_match_plain(bits):
    """Batches of a single job (the smallest runs of the executor): every op
    (and order flags) at N = 2^6, 2^10, 2^14, 2^17, against the plain entry
    points, repeated runs, sampled outputs to the oracle."""
    require_gpu()
    import torch
    limbs = W.limbs_for_bits(bits)
    g = W.rng(9500 + bits)
    for log2n in (6, 10, 14, 17):
        for op in (mwntt.NTT_JOB_FORWARD, mwntt.NTT_JOB_INVERSE, mwntt.NTT_JOB_POLYMUL):
            flags = 0
            if op == mwntt.NTT_JOB_FORWARD and log2n == 14:
                flags = mwntt.NTT_BITREV_OUT
            if op == mwntt.NTT_JOB_INVERSE and log2n == 10:
                flags = mwntt.NTT_BITREV_IN
            q = prime(bits, 70 + log2n % 3)
            plan = mwntt.ntt_plan(log2n, q, limbs, flags=flags)
            n = plan.n
            A, B = W.uniform_residues(g, q, n, limbs), W.uniform_residues(g, q, n, limbs)
            a, b = dev(A), dev(B)
            out = torch.empty_like(a)
            batch = mwntt.NttBatch([(plan, op, a, b if op == mwntt.NTT_JOB_POLYMUL else None, out)])
            announce("single job", bits, log2n, op, flags, batch.info())
            want = _plain(plan, op, a, b)
            for rep in range(2):
                out.zero_()
                batch.run()
                batch.check()
                assert torch.equal(out, want), f"N 2^{log2n} op {op} flags {flags} run {rep}"
            if log2n <= 10:
                ks = [0, n - 1, (log2n * 37) % n]
                got = host_ints(out, limbs)
                a_i, b_i = W.to_ints(A), W.to_ints(B)
                if op == mwntt.NTT_JOB_POLYMUL:
                    assert [got[k] for k in ks] == oracle.polymul.negacyclic_at(a_i, b_i, q, ks)
                elif op == mwntt.NTT_JOB_FORWARD:
                    pos = [bitrev(k, log2n) if flags & mwntt.NTT_BITREV_OUT else k for k in ks]
                    assert [got[p_] for p_ in pos] == oracle.ntt.forward_at(a_i, q, ks)
            batch.destroy()
            plan.destroy()


def test_edge_width_jobs_match_plain():
    """Executor jobs at the low ends of the width classes: products (point-wise
    Barrett in the fused rows) at 97 and 225 bits, the smallest widths Barrett
    takes in two and four words, and transforms at 61 and 125 bits, in one
    mixed batch and in single-width batches, against the plain entry points."""
    require_gpu()
    import torch
    specs = [(10, 97, mwntt.NTT_JOB_POLYMUL), (14, 97, mwntt.NTT_JOB_POLYMUL), (16, 97, mwntt.NTT_JOB_FORWARD),
             (10, 225, mwntt.NTT_JOB_POLYMUL), (13, 225, mwntt.NTT_JOB_POLYMUL), (12, 125, mwntt.NTT_JOB_INVERSE),
             (15, 61, mwntt.NTT_JOB_FORWARD), (11, 61, mwntt.NTT_JOB_INVERSE), (14, 125, mwntt.NTT_JOB_FORWARD)]
    g = W.rng(9700)
    jobs, refs = [], []
    for k, (log2n, bits, op) in enumerate(specs):
        q = prime(bits, 80 + k % 2)
        limbs = W.limbs_for_bits(bits)
        plan = mwntt.ntt_plan(log2n, q, limbs)
        A, B = W.uniform_residues(g, q, plan.n, limbs), W.uniform_residues(g, q, plan.n, limbs)
        a, b = dev(A), dev(B)
        out = torch.empty_like(a)
        jobs.append((plan, op, a, b if op == mwntt.NTT_JOB_POLYMUL else None, out))
        refs.append((plan, op, a, b, out, A, B))
    groups = [list(range(len(jobs)))] + [[i for i, sp in enumerate(specs) if W.limbs_for_bits(sp[1]) == l]
                                         for l in (2, 4)]
    for gi, idx in enumerate(groups):
        batch = mwntt.NttBatch([jobs[i] for i in idx])
        announce("edge width jobs", gi, batch.info())
        for i in idx:
            refs[i][4].zero_()
        batch.run()
        batch.check()
        for i in idx:
            plan, op, a, b, out, A, B = refs[i]
            assert torch.equal(out, _plain(plan, op, a, b)), f"group {gi} job {i} ({specs[i]})"
            if op == mwntt.NTT_JOB_POLYMUL and plan.n <= 1 << 10:
                ks = [0, plan.n - 1, 321]
                got = host_ints(out, plan.limbs)
                assert [got[k] for k in ks] == oracle.polymul.negacyclic_at(W.to_ints(A), W.to_ints(B), plan.q, ks)
        batch.destroy()
    for plan, *_ in refs:
        plan.destroy()


# Odd widths across the three classes for the fused products (point-wise
# Barrett on the scaled modulus): 12289 (14 bits, q = 1 mod 2^12) and 65537
# (17 bits, q = 1 mod 2^16) written out, the rest seeded primes.
PRODUCT_WIDTHS = [14, 17, 33, 59, 61, 80, 96, 97, 123, 125, 160, 200, 224, 225, 251]


def _product_modulus(bits):
    return {14: 12289, 17: 65537}.get(bits) or prime(bits, 900 + bits)


def test_products_every_width():
    """Fused negacyclic products at every width-class position, one mixed
    batch (N = 2^6 .. 2^8 whole outputs against the oracle's schoolbook
    product), then each job again as a batch of its own (kernel-argument
    path) against the same outputs."""
    require_gpu()
    import torch
    jobs, checks, plans = [], [], []
    for k, bits in enumerate(PRODUCT_WIDTHS):
        q = _product_modulus(bits)
        limbs = W.limbs_for_bits(bits)
        log2n = 6 + k % 3
        plan = mwntt.ntt_plan(log2n, q, limbs)
        plans.append(plan)
        g = W.rng(9900 + bits)
        A, B = W.uniform_residues(g, q, plan.n, limbs), W.uniform_residues(g, q, plan.n, limbs)
        a, b = dev(A), dev(B)
        out = torch.empty_like(a)
        jobs.append((plan, mwntt.NTT_JOB_POLYMUL, a, b, out))
        checks.append((out, limbs, oracle.polymul.negacyclic(W.to_ints(A), W.to_ints(B), q), bits))
    batch = mwntt.NttBatch(jobs)
    announce("products every width", batch.info())
    batch.run()
    batch.check()
    for out, limbs, want, bits in checks:
        assert host_ints(out, limbs) == want, f"{bits}-bit product"
    batch.destroy()
    for job, (out, limbs, want, bits) in zip(jobs, checks):
        announce("single product", bits)
        out.zero_()
        one = mwntt.NttBatch([job])
        one.run()
        one.check()
        assert host_ints(out, limbs) == want, f"{bits}-bit product, single job"
        one.destroy()
    for plan in plans:
        plan.destroy()
