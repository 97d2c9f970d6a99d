"""Benchmark of the multi-word NTT / modular BLAS hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--legs all|none|LEG,...]

Workload (one step, the paper-scale plain configuration): forward and inverse
negacyclic NTT at N = 2^16 over a 124-bit prime q = 1 mod 2^18 (coefficients
uniform in [0, q), two 64-bit limbs), then vec_mulmod, vec_addmod and
vec_axpymod on length-2^16 vectors, one library call per operation.  Inputs are
seeded synthetic data already resident in device memory.

Prints one JSON line.  ``value`` is 124-bit NTTs per second of the whole step
(2 transforms per step).  Extra fields: the host issue time per step and the
same step replayed from a hipGraph; per-op latency p50/p99 (HIP events on the
op's stream); algorithmic Gmulmod/s; the batched (96 transforms per call)
rate; ``legs``: the executor on the same batch, a batch sweep, a
host-inclusive (pinned copies in and out) figure, the mixed 96-polynomial
batch and its inverse, 256 fused products at 2^14, RNS products over eight
primes, the 60-bit and 252-bit transforms and BLAS, BLAS at streaming sizes
(2^24) against the HBM peak with both products of vec_mulmod (schoolbook and
Karatsuba), the arithmetic variants of the 124-bit butterfly (the GPU analog
of the paper's MQX ablation), and the serving replay (host-scheduled slots and
the device-resident loop); the roofline of the dominant kernel (with HBM
traffic and VALU instructions from the committed rocprofv3 summary); the CPU
oracle's rate on a bounded sample; and ``cpu_ref``, the scalar C++ baseline
(unsigned __int128 double-words) on one core and on up to 16 cores.  --legs
selects the legs after the plain step (the profiling commands run one leg).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X peaks (published): HBM3E 8 TB/s; 256 CUs x 4 SIMD16 x 2.4 GHz = 39.3 T
# 32-bit integer VALU lane-ops/s.
HBM_PEAK_GBS = 8000.0
INT32_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12

# Algorithmic 32-bit word operations per butterfly (schoolbook Shoup mul-mod
# with W words: quotient estimate from the W(W+1)/2 top-column partial
# products, W(W+1)/2 each for the low halves of x*w and Q*q, W word subs for
# the remainder, and 2W word add/sub for the butterfly's sum and difference).
PROFILE = os.path.join(ROOT, "profiles", "ntt_fwd_2e16_124bit_b64.md")
KERNEL_SOURCES = ["mw_arith.h", "mw_butterfly.h", "mw_ntt_tile.h", "mw_ntt_kernels.inc", "mw_ntt.hip", "mw_tuned.h"]
LEGS = ("batched", "sweep", "host", "mixed", "fused", "rns", "w60", "w252", "blas", "serving", "ablation", "cpu_ref",
        "roofline")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2509_12494_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _profile_value(key):
    """A `- key: value` line of the committed rocprofv3 summary, or None when
    the summary is missing or the kernel sources changed since it was taken."""
    try:
        lines = open(PROFILE).read().splitlines()
    except OSError:
        return None
    kv = dict(l.split(":", 1) for l in lines if l.startswith("- ") and ":" in l)
    kv = {k[2:].strip(): v.strip() for k, v in kv.items()}
    if kv.get("source_hash") != kernel_source_hash():
        return None
    v = kv.get(key)
    return int(v) if v else None


def measured_traffic(pass_):
    """HBM bytes per launch of the pass (FETCH_SIZE + WRITE_SIZE scaled by a
    copy of known size)."""
    return _profile_value(f"traffic_bytes_pass{pass_}")


def measured_valu(pass_):
    """VALU wave-instructions per launch of the pass (SQ_INSTS_VALU)."""
    return _profile_value(f"valu_insts_pass{pass_}")


def butterfly_word_ops(W):
    return 3 * (W * (W + 1) // 2) + W + 2 * W


# The planning model of 32-bit word operations per butterfly that the roofline
# fraction is reported against: about 36 word multiplies and 64 other
# operations for a two-word (124-bit) residue, 10 and 24 for one word.
MODEL_OPS_PER_BUTTERFLY = {4: 100, 2: 34}


def percentile(xs, p):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * p / 100.0
    lo, hi = int(k), min(int(k) + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def progress(msg):
    """Progress on stderr (the JSON result is the only stdout line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def time_calls(fn, stream, reps=20, warm=3, warm_s=0.03):
    """Mean microseconds per call of fn() on `stream` (HIP events), after at
    least `warm` calls and `warm_s` seconds of calls: the first calls of a
    kernel after other work or idling ran up to 23% slower (252-bit
    vec_mulmod at 2^23: 160.9 vs 130.7 us), which the steady state does not."""
    import torch
    t0 = time.perf_counter()
    done = 0
    while done < warm or time.perf_counter() - t0 < warm_s:
        fn()
        done += 1
        if done % 8 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e3 / reps


def time_graph(fn, stream, reps=20):
    """Capture fn(stream) into a hipGraph, then mean microseconds per replay."""
    import torch
    s = torch.cuda.Stream()
    fn(s.cuda_stream)            # eager warm-up on the capture stream
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        fn(s.cuda_stream)
    torch.cuda.synchronize()
    us = time_calls(g.replay, torch.cuda.current_stream(), reps=reps)
    del g
    return us


def serving_leg(count, rate=20000.0, budget=1 << 30, spin_us=0, modes=("slots", "resident", "resident_spin")):
    """Open-loop Poisson stream through the serving runtime (inputs pre-staged),
    once per scheduling mode: "slots" (the host scheduler launches each batch
    on a stream), "resident" (the device-resident request loop) and
    "resident_spin" (the loop with a scheduler that polls without sleeping,
    spin_us = 1000: one busy host core).

    70% transforms (half forward, half inverse) with N = 2^e, e uniform in
    10..17; 30% BLAS (half mulmod, half axpymod) with length floor(2^u), u
    uniform in [10, 17]; 60- or 124-bit moduli with equal probability."""
    import torch
    from paper_2509_12494_amd import mwntt
    from paper_2509_12494_amd import workloads as W
    jobs = W.serving_stream(count, rate=rate, primes_per_width=2)
    plans, bufs = {}, {}

    def buf(q, limbs, n, tag):
        key = (q, n, tag)
        if key not in bufs:
            bufs[key] = mwntt.to_device(W.uniform_residues(W.rng(len(bufs) + 77), q, n, limbs))
        return bufs[key]

    reqs, arrivals = [], []
    for j in jobs:
        q, limbs, op = j["q"], j["limbs"], j["op"]
        if op.startswith("ntt"):
            lg = j["size"].bit_length() - 1
            if (lg, q) not in plans:
                plans[(lg, q)] = mwntt.ntt_plan(lg, q, limbs)
            plan = plans[(lg, q)]
            code = mwntt.MW_REQ_NTT_FORWARD if op == "ntt_forward" else mwntt.MW_REQ_NTT_INVERSE
            reqs.append(mwntt.make_request(code, buf(q, limbs, j["size"], "a"), plan=plan))
        else:
            code = mwntt.MW_REQ_VEC_MULMOD if op == "vec_mulmod" else mwntt.MW_REQ_VEC_AXPYMOD
            a, b = buf(q, limbs, 1 << 17, "a"), buf(q, limbs, 1 << 17, "b")
            reqs.append(mwntt.make_request(code, a, b, q=q, limbs=limbs, n=j["size"], alpha=(q - 1) // 3))
        arrivals.append(j["t"] * 1e6)
    torch.cuda.synchronize()
    progress(f"serving: {len(plans)} plans, {len(bufs)} input buffers staged")
    out = {"requests": count, "offered_rate": rate, "hbm_budget": budget, "spin_us": spin_us}
    for mode in modes:
        srv = mwntt.MwServer(budget, max_inflight=4, max_batch=64, spin_us=1000 if mode == "resident_spin" else spin_us,
                             resident=mode.startswith("resident"))
        warm = min(2000, count)
        srv.replay(reqs[:warm], [a - arrivals[0] for a in arrivals[:warm]])
        lat, span = srv.replay(reqs, arrivals)
        st = srv.stats()
        srv.destroy()
        out[mode] = {"throughput_req_s": round(count / (span * 1e-6), 1),
                     "p50_us": round(percentile(lat, 50), 2), "p99_us": round(percentile(lat, 99), 2),
                     "mean_us": round(sum(lat) / len(lat), 2), "makespan_s": round(span * 1e-6, 4),
                     "batches": st["batches"], "max_batch": st["max_batch_seen"], "pool_peak_bytes": st["pool_peak"],
                     "resident_requests": st["resident_requests"], "resident_launches": st["resident_launches"]}
        progress(f"serving ({mode}): p50 {out[mode]['p50_us']} us, p99 {out[mode]['p99_us']} us")
    for p in plans.values():
        p.destroy()
    return out


def cpu_baseline(wl, budget_s=12.0):
    """The oracle (plain Python integers, one core) on a bounded sample of the
    same workload: forward-NTT outputs of the 2^16-point polynomial computed one
    by one from the definition, scaled to whole transforms per second."""
    import oracle
    from paper_2509_12494_amd import workloads as W
    a = W.to_ints(wl.data["poly"])
    n = len(a)
    t0 = time.perf_counter()
    done = 0
    k = 0
    while time.perf_counter() - t0 < budget_s:
        oracle.ntt.forward_at(a, wl.q, [k])
        done += 1
        k = (k * 7919 + 1) % n
    dt = time.perf_counter() - t0
    per_output = dt / done
    return {"value": 1.0 / (per_output * n), "unit": "NTT/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} forward outputs A_k of one N=2^16 124-bit transform, each an O(N) sum "
                      f"from the definition ({dt:.1f} s), scaled to N outputs per transform"}


def cpu_ref_leg(wl, budget_s=1.5):
    """The scalar C++ baseline (cpu_ref: unsigned __int128 double-words,
    schoolbook products, Barrett) on the same 2^16 124-bit polynomial: forward
    transforms on one core and on every core this process may use (at most 16,
    the host share of one GPU), and 124-bit vec_mulmod over 2^22 residues."""
    import numpy as np
    import cpu_ref
    from paper_2509_12494_amd import workloads as W
    threads = min(16, len(os.sched_getaffinity(0)))
    q, limbs, log2n = wl.q, wl.limbs, wl.log2n
    poly = np.ascontiguousarray(wl.data["poly"], dtype=np.uint64)
    plan = cpu_ref.Plan(log2n, q, limbs)

    def rate(fn, units):
        fn()                                      # warm
        done, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < budget_s:
            fn()
            done += units
        return done / (time.perf_counter() - t0)

    ntt_1 = rate(lambda: plan.transform(poly, threads=1), 1)
    batch = np.concatenate([poly] * (2 * threads))
    ntt_all = rate(lambda: plan.transform(batch, threads=threads), 2 * threads)
    x = W.uniform_residues(W.rng(91), q, 1 << 22, limbs)
    y = W.uniform_residues(W.rng(92), q, 1 << 22, limbs)
    mul_1 = rate(lambda: cpu_ref.blas("mul", x, y, q, limbs, threads=1), 1 << 22)
    mul_all = rate(lambda: cpu_ref.blas("mul", x, y, q, limbs, threads=threads), 1 << 22)
    plan.destroy()
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return {"kind": "cpu_ref (scalar C++, unsigned __int128 double-words, schoolbook + Barrett, g++ -O3)",
            "cpu": model, "threads_all": threads,
            "workload": "forward negacyclic NTT N=2^16, 124-bit q (the plain step's); vec_mulmod n=2^22, 124-bit",
            "ntt_s_1core": round(ntt_1, 2), "ntt_s_all": round(ntt_all, 2),
            "gmulmod_s_1core": round(mul_1 / 1e9, 4), "gmulmod_s_all": round(mul_all / 1e9, 4)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200,
                    help="timed steps (200: the 1400 launches fit in the device queue, so the host never waits for a free slot)")
    ap.add_argument("--warmup", type=int, default=2000,
                    help="untimed steps before the timed ones (2000 steps, about 60 ms: the clocks settle)")
    ap.add_argument("--batch", type=int, default=96, help="transforms per call in the batched leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=100000,
                    help="requests in the serving leg (Poisson, 20k requests/s); 0 skips it")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run one device-to-device copy of this many MiB (counter calibration)")
    ap.add_argument("--legs", default="all",
                    help="comma-separated legs after the plain step (" + ",".join(LEGS) + "), 'all' or 'none'")
    args = ap.parse_args()
    legs_on = set(LEGS) if args.legs == "all" else set(x for x in args.legs.split(",") if x and x != "none")
    unknown = legs_on - set(LEGS)
    if unknown:
        print(f"unknown legs: {sorted(unknown)}", file=sys.stderr)
        sys.exit(2)
    if args.gpus != 1:
        print("bench.py measures one GPU; runs on more than one GPU are not supported", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2509_12494_amd import mwntt
    from paper_2509_12494_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    wl = W.config_paper(124)
    q, limbs, log2n = wl.q, wl.limbs, wl.log2n
    n = 1 << log2n
    plan = mwntt.ntt_plan(log2n, q, limbs)
    poly = mwntt.to_device(wl.data["poly"])
    spec = torch.empty_like(poly)
    back = torch.empty_like(poly)
    xa = mwntt.to_device(wl.data["a"])
    xb = mwntt.to_device(wl.data["b"])
    c_mul = torch.empty_like(xa)
    c_add = torch.empty_like(xa)
    y = xb.clone()
    alpha = wl.data["alpha"]
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream

    ops = {
        "ntt_forward": lambda: plan.forward(spec, poly, batch=1, stream=sp),
        "ntt_inverse": lambda: plan.inverse(back, spec, batch=1, stream=sp),
        "vec_mulmod": lambda: mwntt.vec_mulmod(c_mul, xa, xb, q, limbs, stream=sp),
        "vec_addmod": lambda: mwntt.vec_addmod(c_add, xa, xb, q, limbs, stream=sp),
        "vec_axpymod": lambda: mwntt.vec_axpymod(y, alpha, xa, q, limbs, stream=sp),
    }

    def step():
        for f in ops.values():
            f()

    progress("plain step")
    # untimed steps; a synchronize every 100 keeps the device queue from
    # filling (a host that waits for free queue slots issues slower after)
    for i in range(args.warmup):
        step()
        if i % 100 == 99:
            torch.cuda.synchronize()
    torch.cuda.synchronize()

    # timed region: exactly K steps
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    t_enq = time.perf_counter() - t0       # host time to issue the K steps
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = ev0.elapsed_time(ev1)
    ms_per_step = ms_total / args.steps

    # correctness of the timed outputs: the inverse undid the forward
    assert torch.equal(back, poly), "round trip failed"

    # the same step with its 7 launches captured once in a hipGraph and
    # replayed: one launch per op as above, without the per-call host work
    gstream = torch.cuda.Stream()
    gsp = gstream.cuda_stream
    gops = [lambda: plan.forward(spec, poly, batch=1, stream=gsp),
            lambda: plan.inverse(back, spec, batch=1, stream=gsp),
            lambda: mwntt.vec_mulmod(c_mul, xa, xb, q, limbs, stream=gsp),
            lambda: mwntt.vec_addmod(c_add, xa, xb, q, limbs, stream=gsp),
            lambda: mwntt.vec_axpymod(y, alpha, xa, q, limbs, stream=gsp)]
    for f in gops:
        f()
    torch.cuda.synchronize()
    sgraph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(sgraph, stream=gstream):
        for f in gops:
            f()
    torch.cuda.synchronize()
    graph_us = time_calls(sgraph.replay, torch.cuda.current_stream(), reps=args.steps)
    back.zero_()
    sgraph.replay()
    torch.cuda.synchronize()
    assert torch.equal(back, poly), "graph-replayed round trip failed"
    del sgraph

    # per-op latency, each op bracketed by events on its stream (paper protocol:
    # mean of the last half of the runs; here also p50 / p99)
    lat = {}
    for name, f in ops.items():
        reps = 200
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for e0, e1 in evs:
            e0.record(stream)
            f()
            e1.record(stream)
        torch.cuda.synchronize()
        us = [e0.elapsed_time(e1) * 1e3 for e0, e1 in evs]
        half = us[reps // 2:]
        lat[name] = {"p50_us": round(percentile(us, 50), 3), "p99_us": round(percentile(us, 99), 3),
                     "mean_last_half_us": round(sum(half) / len(half), 3)}

    # the batch of 2^16 transforms several legs use (same plan, same q)
    B = args.batch
    bpoly = mwntt.to_device(W.uniform_residues(W.rng(2100), q, n * B, limbs))
    bspec = torch.empty_like(bpoly)
    legs = {}
    batched_us = batched_ntt_s = None
    if "batched" in legs_on:
        progress("batched legs")
        # batched leg: many 2^16 transforms in one call
        batched_us = time_calls(lambda: plan.forward(bspec, bpoly, batch=B, stream=sp), stream)
        batched_ntt_s = B / (batched_us * 1e-6)
        # the same 96 transforms through the batched executor, replayed from a graph
        ex = mwntt.NttBatch([(plan, mwntt.NTT_JOB_FORWARD, bpoly[i * n:(i + 1) * n], None,
                              bspec[i * n:(i + 1) * n]) for i in range(B)])
        exec_us = time_graph(lambda s_: ex.run(stream=s_), stream)
        legs["homogeneous_2e16"] = {"batch": B, "ntt_forward_us_per_call": round(batched_us, 2),
                                    "ntt_forward_ntt_s": round(batched_ntt_s, 1),
                                    "executor_graph_us": round(exec_us, 2),
                                    "executor_ntt_s": round(B / (exec_us * 1e-6), 1)}
        ex.destroy()

    # batch sweep of the same transform (inputs: the 96 staged polynomials
    # repeated, all canonical residues)
    if "sweep" in legs_on:
        sweep_leg(plan, bpoly, B, n, stream, sp, legs)
    if "host" in legs_on:
        host_leg(plan, poly, spec, bpoly, bspec, B, n, limbs, stream, sp, legs)
    if "mixed" in legs_on:
        mixed_leg(stream, sp, legs)
    if "fused" in legs_on:
        fused_leg(stream, legs)
    if "rns" in legs_on:
        rns_leg(n, stream, legs)
    if "w60" in legs_on:
        w60_leg(n, stream, sp, legs)
    if "w252" in legs_on:
        w252_leg(n, log2n, stream, sp, legs)
    if "blas" in legs_on:
        blas_leg(stream, sp, legs)
    if "ablation" in legs_on:
        ablation_leg(q, n, bpoly, bspec, B, stream, sp, legs)
    if args.serve_requests and "serving" in legs_on:
        progress(f"serving leg: {args.serve_requests} requests")
        legs["serving"] = serving_leg(args.serve_requests)

    roof = roofline_leg(plan, bpoly, bspec, B, n, log2n, limbs, stream, sp) if "roofline" in legs_on else None

    mulmods_step = 2 * bfly_count(n, log2n) + 2 * n        # two transforms + vec_mulmod + vec_axpymod
    res = {
        "metric": "128-bit NTT/s at N=2^16 (batched vs plain), Gmulmod/s, p50/p99 latency",
        "value": round(2.0 / (ms_per_step * 1e-3), 2),
        "unit": "NTT/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u128 (2x64-bit limbs, 124-bit prime)",
        "data": "synthetic (seeded uniform residues)",
        "config": {"workload": "plain, paper scale: forward+inverse negacyclic NTT N=2^16, 124-bit q=1 mod 2^18; "
                               "vec_mulmod/addmod/axpymod n=2^16; one launch per op",
                   "N": n, "q_bits": q.bit_length(), "limbs": limbs, "split_log_n1": plan.split},
        "gmulmod_s": round(mulmods_step / (ms_per_step * 1e-3) / 1e9, 4),
        "latency_us": lat,
        "batched": None if batched_us is None else {
            "batch": B, "us_per_call": round(batched_us, 2), "ntt_s": round(batched_ntt_s, 1),
            "speedup_vs_plain_forward": round(batched_ntt_s / (1e6 / lat["ntt_forward"]["p50_us"]), 2),
            "gmulmod_s": round(B * bfly_count(n, log2n) / (batched_us * 1e-6) / 1e9, 3)},
        "legs": legs,
        "roofline": roof,
        "wall_s_timed_region": round(wall, 4),
        # host time to issue one step (7 library calls through the Python
        # binding); close to ms_per_step means the plain step is bound by
        # call submission rather than by the GPU
        "host_issue_us_per_step": round(t_enq / args.steps * 1e6, 2),
        "plain_step_graph": {"us_per_step": round(graph_us, 2), "ntt_s": round(2.0 / (graph_us * 1e-6), 1),
                             "note": "the same step (7 launches, one per op) captured once in a hipGraph"},
    }
    if args.copy_calibration_mib:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE readings scale
        # the counters of the transform kernels to bytes
        nbytes = args.copy_calibration_mib << 20
        src = torch.empty(nbytes // 8, dtype=torch.int64, device="cuda").fill_(3)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        res["copy_calibration_bytes"] = nbytes
    if not args.no_cpu_baseline:
        progress("cpu baseline (oracle)")
        res["cpu_baseline"] = cpu_baseline(wl)
        if "cpu_ref" in legs_on:
            progress("cpu_ref (scalar C++ baseline)")
            cr = cpu_ref_leg(wl)
            cr["gpu_plain_over_1core"] = round(res["value"] / cr["ntt_s_1core"], 1)
            if batched_ntt_s:
                cr["gpu_batched_over_all"] = round(batched_ntt_s / cr["ntt_s_all"], 1)
            res["cpu_ref"] = cr
    plan.destroy()
    print(json.dumps(res), flush=True)


def bfly_count(n, log2n):
    return (n // 2) * log2n


def sweep_leg(plan, bpoly, B, n, stream, sp, legs):
    import torch
    progress("batch sweep")
    sweep_max = 1024
    reps_in = (sweep_max + B - 1) // B
    sw_in = bpoly.repeat(reps_in, 1)[:sweep_max * n]
    sw_out = torch.empty_like(sw_in)
    sweep = {}
    for bs in (1, 8, 32, 96, 256, 1024):
        us = time_calls(lambda: plan.forward(sw_out, sw_in, batch=bs, stream=sp), stream, reps=10 if bs >= 256 else 20)
        sweep[str(bs)] = {"us_per_call": round(us, 2), "ntt_s": round(bs / (us * 1e-6), 1)}
    legs["batch_sweep_2e16"] = sweep
    del sw_in, sw_out


def host_leg(plan, poly, spec, bpoly, bspec, B, n, limbs, stream, sp, legs):
    """Host-inclusive form (the paper's CPU timings include data transfer):
    pinned host input -> device, forward transform, device -> pinned host."""
    import torch
    progress("host-inclusive")
    h_in = torch.empty(poly.shape, dtype=poly.dtype, pin_memory=True)
    h_in.copy_(poly)
    h_out = torch.empty_like(h_in, pin_memory=True)
    d_in = torch.empty_like(poly)
    d_out = torch.empty_like(poly)

    def host_round():
        d_in.copy_(h_in, non_blocking=True)
        plan.forward(d_out, d_in, batch=1, stream=sp)
        h_out.copy_(d_out, non_blocking=True)
    host_us = time_calls(host_round, stream)
    torch.cuda.synchronize()
    want = torch.empty_like(poly)
    plan.forward(want, poly, batch=1, stream=sp)
    torch.cuda.synchronize()
    assert torch.equal(h_out, want.cpu()), "host-inclusive forward differs"
    hb_in = torch.empty(bpoly.shape, dtype=bpoly.dtype, pin_memory=True)
    hb_in.copy_(bpoly)
    hb_out = torch.empty_like(hb_in, pin_memory=True)

    def host_round_b():
        bpoly.copy_(hb_in, non_blocking=True)
        plan.forward(bspec, bpoly, batch=B, stream=sp)
        hb_out.copy_(bspec, non_blocking=True)
    host_b_us = time_calls(host_round_b, stream, reps=10)
    legs["host_inclusive_2e16"] = {"ntt_forward_us": round(host_us, 2), "ntt_s": round(1 / (host_us * 1e-6), 1),
                                   "batch": B, "batched_us": round(host_b_us, 2),
                                   "batched_ntt_s": round(B / (host_b_us * 1e-6), 1),
                                   "bytes_per_transform": 2 * n * 8 * limbs}


def mixed_leg(stream, sp, legs):
    """Mixed batch: 96 polynomials, N uniform over 2^12..2^16, 60/124-bit,
    forward (and the inverse batch of the round trip)."""
    import torch
    from paper_2509_12494_amd import mwntt
    from paper_2509_12494_amd import workloads as W
    progress("mixed batch")
    mixed = W.config_batched()
    mplans, mjobs, mbfly = {}, [], 0
    for (lg, qm, lm, coeffs) in mixed:
        if (lg, qm) not in mplans:
            mplans[(lg, qm)] = mwntt.ntt_plan(lg, qm, lm)
        pl = mplans[(lg, qm)]
        x = mwntt.to_device(coeffs)
        mjobs.append((pl, mwntt.NTT_JOB_FORWARD, x, None, torch.empty_like(x)))
        mbfly += (1 << (lg - 1)) * lg
    mb = mwntt.NttBatch(mjobs)
    mixed_us = time_graph(lambda s_: mb.run(stream=s_), stream)
    mb.run(stream=sp)
    ijobs = [(pl, mwntt.NTT_JOB_INVERSE, o, None, torch.empty_like(o)) for (pl, _, _, _, o) in mjobs]
    mi = mwntt.NttBatch(ijobs)
    mi.run(stream=sp)
    torch.cuda.synchronize()
    for (_, _, x, _, _), (_, _, _, _, r) in zip(mjobs, ijobs):
        assert torch.equal(x, r), "mixed round trip failed"
    mixed_inv_us = time_graph(lambda s_: mi.run(stream=s_), stream)
    mi.destroy()
    legs["mixed_96"] = {"polys": len(mixed), "us_per_run": round(mixed_us, 2),
                        "inverse_us_per_run": round(mixed_inv_us, 2),
                        "polys_s": round(len(mixed) / (mixed_us * 1e-6), 1),
                        "gbutterfly_s": round(mbfly / (mixed_us * 1e-6) / 1e9, 2)}
    mb.destroy()
    for pl in mplans.values():
        pl.destroy()


def fused_leg(stream, legs):
    """Fused products: 256 pairs at N = 2^14, 124-bit, one executor run
    replayed from a hipGraph."""
    import torch
    from paper_2509_12494_amd import mwntt
    from paper_2509_12494_amd import workloads as W
    progress("fused products")
    qf, FA, FB = W.config_fused()
    pairs, nf = FA.shape[0], FA.shape[1]
    fplan = mwntt.ntt_plan(14, qf, 2)
    fa, fb = mwntt.to_device(FA.reshape(-1, 2)), mwntt.to_device(FB.reshape(-1, 2))
    fc = torch.empty_like(fa)
    fbatch = mwntt.NttBatch([(fplan, mwntt.NTT_JOB_POLYMUL, fa[i * nf:(i + 1) * nf], fb[i * nf:(i + 1) * nf],
                              fc[i * nf:(i + 1) * nf]) for i in range(pairs)])
    fused_us = time_graph(lambda s_: fbatch.run(stream=s_), stream)
    legs["fused_256x2e14"] = {"pairs": pairs, "us_per_run": round(fused_us, 2),
                              "products_s": round(pairs / (fused_us * 1e-6), 1),
                              "ntt_equiv_s": round(3 * pairs / (fused_us * 1e-6), 1)}
    fbatch.destroy()
    fplan.destroy()


def rns_leg(n, stream, legs):
    """RNS form (the FHE shape): polynomials mod Q = q_1 ... q_8, eight 124-bit
    primes sharing N = 2^16; 4 RNS products = 32 fused product jobs in one
    executor run (hipGraph replay)."""
    import torch
    from paper_2509_12494_amd import mwntt
    from paper_2509_12494_amd import workloads as W
    progress("rns leg")
    rqs = W.config_rns()
    rplans = [mwntt.ntt_plan(16, rq, 2) for rq in rqs]
    rpolys = 4
    rjobs = []
    for j in range(rpolys):
        for i, rq in enumerate(rqs):
            ra = mwntt.to_device(W.uniform_residues(W.rng(7200 + 16 * j + i), rq, n, 2))
            rb = mwntt.to_device(W.uniform_residues(W.rng(7300 + 16 * j + i), rq, n, 2))
            rjobs.append((rplans[i], mwntt.NTT_JOB_POLYMUL, ra, rb, torch.empty_like(ra)))
    rbatch = mwntt.NttBatch(rjobs)
    rns_us = time_graph(lambda s_: rbatch.run(stream=s_), stream)
    legs["rns_8x124bit_2e16"] = {"moduli": len(rqs), "q_bits": 124, "N": n, "rns_products": rpolys,
                                 "us_per_run": round(rns_us, 2),
                                 "rns_products_s": round(rpolys / (rns_us * 1e-6), 1),
                                 "residue_products_s": round(len(rjobs) / (rns_us * 1e-6), 1)}
    rbatch.destroy()
    for pl in rplans:
        pl.destroy()


def w60_leg(n, stream, sp, legs):
    """The paper-scale transform with a 60-bit prime (one word): plain
    latency, 96 per call, mulmod."""
    import torch
    from paper_2509_12494_amd import mwntt
    from paper_2509_12494_amd import workloads as W
    progress("60-bit leg")
    q1 = W.find_prime(60, 2001)
    p60 = mwntt.ntt_plan(16, q1, 1)
    x60 = mwntt.to_device(W.uniform_residues(W.rng(6050), q1, n * 96, 1))
    y60, z60 = torch.empty_like(x60), torch.empty_like(x60)
    p60.forward(y60, x60, batch=96, stream=sp)
    p60.inverse(z60, y60, batch=96, stream=sp)
    torch.cuda.synchronize()
    assert torch.equal(z60, x60), "60-bit round trip failed"
    b60_us = time_calls(lambda: p60.forward(y60, x60, batch=96, stream=sp), stream, reps=10)
    x1, y1, z1, x2 = x60[:n], y60[:n], z60[:n], x60[n:2 * n]
    legs["plain_60bit_2e16"] = {
        "q_bits": 60, "N": n,
        "ntt_forward_us": round(time_calls(lambda: p60.forward(y1, x1, batch=1, stream=sp), stream, reps=50), 2),
        "ntt_inverse_us": round(time_calls(lambda: p60.inverse(z1, y1, batch=1, stream=sp), stream, reps=50), 2),
        "batch": 96, "batched_us_per_call": round(b60_us, 2), "batched_ntt_s": round(96 / (b60_us * 1e-6), 1),
        "vec_mulmod_us": round(time_calls(lambda: mwntt.vec_mulmod(z1, x1, x2, q1, 1, stream=sp), stream, reps=50), 2)}
    p60.destroy()


def w252_leg(n, log2n, stream, sp, legs):
    """Four-word moduli (252-bit q = 1 mod 2^18): N = 2^16, plain latency,
    batch-64 throughput and the BLAS ops, inputs resident in HBM."""
    import torch
    from paper_2509_12494_amd import mwntt
    from paper_2509_12494_amd import workloads as W
    progress("252-bit leg")
    q8 = W.find_prime(252, 6001)
    wplan = mwntt.ntt_plan(16, q8, 4)
    wb = 64
    wx = mwntt.to_device(W.uniform_residues(W.rng(6100), q8, n * wb, 4))
    wy, wz = torch.empty_like(wx), torch.empty_like(wx)
    wplan.forward(wy, wx, batch=wb, stream=sp)
    wplan.inverse(wz, wy, batch=wb, stream=sp)
    torch.cuda.synchronize()
    assert torch.equal(wz, wx), "252-bit round trip failed"
    w1x, w1y = wx[:n], torch.empty_like(wx[:n])
    wide = {"q_bits": 252, "N": n,
            "ntt_forward_us": round(time_calls(lambda: wplan.forward(w1y, w1x, batch=1, stream=sp), stream, reps=50), 2),
            "ntt_inverse_us": round(time_calls(lambda: wplan.inverse(w1y, w1x, batch=1, stream=sp), stream, reps=50), 2)}
    wb_us = time_calls(lambda: wplan.forward(wy, wx, batch=wb, stream=sp), stream, reps=10)
    wide.update({"batch": wb, "batched_us_per_call": round(wb_us, 2), "batched_ntt_s": round(wb / (wb_us * 1e-6), 1),
                 "batched_gbutterfly_s": round(wb * (n // 2) * log2n / (wb_us * 1e-6) / 1e9, 2)})
    wa, wbv = wx[:n], wx[n:2 * n]
    wc = torch.empty_like(wa)
    for nm, f in (("vec_mulmod_us", lambda: mwntt.vec_mulmod(wc, wa, wbv, q8, 4, stream=sp)),
                  ("vec_addmod_us", lambda: mwntt.vec_addmod(wc, wa, wbv, q8, 4, stream=sp))):
        wide[nm] = round(time_calls(f, stream, reps=50), 2)
    legs["wide_252bit_2e16"] = wide
    wplan.destroy()


def blas_leg(stream, sp, legs):
    """BLAS at streaming sizes: n = 2^24 residues (2^23 for 252-bit), inputs
    resident; algorithmic bytes = two vectors read + one written.  vec_mulmod
    is timed with both products of its Barrett reduction (schoolbook columns,
    Karatsuba, Eq. mulk) and reported with the width's default."""
    import torch
    from paper_2509_12494_amd import mwntt
    from paper_2509_12494_amd import workloads as W
    progress("BLAS streaming leg")
    stream_leg = {}
    for bits, lg in ((60, 24), (124, 24), (252, 23)):
        qs = W.find_prime(bits, 2001)
        ls = W.limbs_for_bits(bits)
        ns = 1 << lg
        sa = mwntt.to_device(W.uniform_residues(W.rng(7700 + bits), qs, ns, ls))
        sb = torch.roll(sa, 1, 0)                      # a permutation of the same uniform residues
        sc = torch.empty_like(sa)
        alpha_s = (qs - 1) // 3
        nbytes = 3 * ns * 8 * ls
        row = {"n": ns}

        def put(nm, us):
            gbs = nbytes / (us * 1e-6) / 1e9
            row[nm] = {"us": round(us, 1), "GBs": round(gbs, 1), "frac_hbm": round(gbs / HBM_PEAK_GBS, 3)}
        put("add", time_calls(lambda: mwntt.vec_addmod(sc, sa, sb, qs, ls, stream=sp), stream, reps=20))
        default = mwntt.get_mulmod_product(ls)
        prods, outs = {}, {}
        for kara in (False, True):
            mwntt.set_mulmod_product(ls, kara)
            prods[kara] = time_calls(lambda: mwntt.vec_mulmod(sc, sa, sb, qs, ls, stream=sp), stream, reps=20)
            torch.cuda.synchronize()
            outs[kara] = sc.clone()
        mwntt.set_mulmod_product(ls, default)
        assert torch.equal(outs[False], outs[True]), "Karatsuba and schoolbook products differ"
        put("mul", prods[default])
        row["mul"]["gmulmod_s"] = round(ns / (prods[default] * 1e-6) / 1e9, 2)
        row["mul"]["product"] = "karatsuba" if default else "schoolbook"
        row["mul_products_us"] = {"schoolbook": round(prods[False], 1), "karatsuba": round(prods[True], 1)}
        put("axpy", time_calls(lambda: mwntt.vec_axpymod(sc, alpha_s, sa, qs, ls, stream=sp), stream, reps=20))
        stream_leg[f"{bits}bit"] = row
        del sa, sb, sc, outs
    legs["blas_stream"] = stream_leg


def ablation_leg(q, n, bpoly, bspec, B, stream, sp, legs):
    """The GPU analog of the paper's MQX ablation: the 2^16 124-bit forward
    transform of the batch with the native butterfly and with its arithmetic
    variants (products from multiply-low / multiply-high, carries by
    compare-and-select, both), all in the variants' one shape (two passes of
    2^8-point lines, 4 points per lane, 4 lines per workgroup)."""
    import torch
    from paper_2509_12494_amd import mwntt
    progress("ablation leg")
    rows, ref = {}, None
    for name, flags in (("native", 0), ("mulhi", mwntt.NTT_ARITH_MULHI), ("cmpcarry", mwntt.NTT_ARITH_CMPCARRY),
                        ("mulhi_cmpcarry", mwntt.NTT_ARITH_MULHI | mwntt.NTT_ARITH_CMPCARRY)):
        p = mwntt.ntt_plan(16, q, 2, flags=flags)
        if not flags:
            p.split = 8
            p.set_tiles(1, 2, 4)
            p.set_tiles(2, 2, 4)
        p.forward(bspec, bpoly, batch=B, stream=sp)
        torch.cuda.synchronize()
        if ref is None:
            ref = bspec.clone()
        assert torch.equal(bspec, ref), f"{name} variant differs from the native arithmetic"
        us = time_calls(lambda: p.forward(bspec, bpoly, batch=B, stream=sp), stream, reps=10)
        p1 = time_calls(lambda: p.forward_pass(1, None, bpoly, B, stream=sp), stream, reps=10)
        p2 = time_calls(lambda: p.forward_pass(2, bspec, None, B, stream=sp), stream, reps=10)
        rows[name] = {"forward_us": round(us, 2), "ntt_s": round(B / (us * 1e-6), 1),
                      "pass1_us": round(p1, 2), "pass2_us": round(p2, 2)}
        p.destroy()
    for name in rows:
        rows[name]["slowdown_vs_native"] = round(rows[name]["forward_us"] / rows["native"]["forward_us"], 3)
    legs["ablation_124bit_2e16"] = {"batch": B, "variants": rows}


def roofline_leg(plan, bpoly, bspec, B, n, log2n, limbs, stream, sp):
    """Roofline of the dominant kernel: the two passes of the batched forward
    transform, each one kernel launch, timed with HIP events on their stream.
    Algorithmic work per butterfly: the planning model of 32-bit word
    operations (MODEL_OPS_PER_BUTTERFLY), beside the minimal count of the
    Shoup butterfly's word products and adds (butterfly_word_ops)."""
    import torch
    progress("roofline passes")
    RB = min(64, B)
    rin, rout = bpoly[:RB * n], bspec[:RB * n]
    ref = torch.empty_like(rin)
    plan.forward(ref, rin, batch=RB, stream=sp)
    plan.forward_pass(1, None, rin, RB, stream=sp)
    plan.forward_pass(2, rout, None, RB, stream=sp)
    torch.cuda.synchronize()
    assert torch.equal(ref, rout), "pass 1 + pass 2 differs from ntt_forward"
    large, split = plan.config_for(RB)
    W_words = 2 * limbs
    model_ops = MODEL_OPS_PER_BUTTERFLY[W_words]
    passes = {}
    for k, (stages, fn) in {1: (split, lambda: plan.forward_pass(1, None, rin, RB, stream=sp)),
                            2: (log2n - split, lambda: plan.forward_pass(2, rout, None, RB, stream=sp))}.items():
        us = time_calls(fn, stream, reps=50)
        bfly = RB * (n // 2) * stages
        tw_bytes = (1 << split if k == 1 else n) * 32 * limbs // 2
        byts = 2 * RB * n * 8 * limbs + tw_bytes
        passes[k] = {"us": us, "butterflies": bfly, "bytes": byts}
    dom = max(passes, key=lambda k: passes[k]["us"])
    d = passes[dom]
    achieved = d["butterflies"] * model_ops / (d["us"] * 1e-6) / 1e12
    achieved_min = d["butterflies"] * butterfly_word_ops(W_words) / (d["us"] * 1e-6) / 1e12
    traffic = measured_traffic(dom)
    valu_insts = measured_valu(dom)
    valu_issue = None
    if valu_insts:
        # what the kernel issues, beside the algorithmic count: VALU
        # wave-instructions x 64 lanes per launch, over the same launch time
        issued = valu_insts * 64 / (d["us"] * 1e-6) / 1e12
        valu_issue = {"valu_insts": valu_insts, "lane_ops_per_butterfly": round(valu_insts * 64 / d["butterflies"], 1),
                      "achieved": round(issued, 3), "frac": round(issued / INT32_PEAK_TOPS, 4)}
    return {"bound": "alu",
            "kernel": f"forward pass {dom} ({'column' if dom == 1 else 'row'} tiles), N=2^16, 124-bit, "
                      f"batch {RB}, one launch ({'large-batch' if large else 'single-transform'} configuration)",
            "achieved": round(achieved, 3), "peak": round(INT32_PEAK_TOPS, 2),
            "unit": "Tint32op/s", "frac": round(achieved / INT32_PEAK_TOPS, 4), "traffic": traffic,
            "ops_per_butterfly": model_ops,
            "minimal": {"ops_per_butterfly": butterfly_word_ops(W_words), "achieved": round(achieved_min, 3),
                        "frac": round(achieved_min / INT32_PEAK_TOPS, 4)},
            "launch_us": round(d["us"], 3), "butterflies": d["butterflies"],
            "valu_issue": valu_issue,
            "algorithmic_bytes": d["bytes"],
            "hbm_gbs_algorithmic": round(d["bytes"] / (d["us"] * 1e-6) / 1e9, 1),
            "passes_us": {str(k): round(v["us"], 3) for k, v in passes.items()}}


if __name__ == "__main__":
    main()
