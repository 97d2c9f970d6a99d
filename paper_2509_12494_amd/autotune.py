"""Autotuner for the NTT decomposition and tile shapes.

For one (N, modulus width, batch) it enumerates the plan configurations the
library accepts -- single-workgroup tiles or each N1 x N2 two-pass split, and
per pass the points per lane (2^1..2^4) and lines per workgroup -- times a
forward + inverse round trip of `batch` transforms with HIP events, and checks
every candidate's output against the first configuration's bit for bit (the
shapes only change the schedule, never the result).  Coordinate search: for
each split the column shape is tuned with the row shape at its default, then
the row shape with the best column shape.

    python -m paper_2509_12494_amd.autotune --log2n 16 --bits 124 --batch 1 64 [--out FILE]

Prints one JSON line per (log2n, bits, batch) with the ranked candidates and
the best configuration.  ``apply(plan, cfg)`` sets a found configuration on a
plan.
"""
from __future__ import annotations

import argparse
import json
import sys

from . import mwntt
from . import workloads as W

LINES = (1, 2, 4, 8, 16, 32)


def apply(plan: mwntt.NttPlan, cfg: dict) -> None:
    plan.split = cfg["split"]
    for name, pass_ in (("full", 0), ("col", 1), ("row", 2)):
        if name in cfg:
            plan.set_tiles(pass_, *cfg[name])


def _valid_shapes(plan, pass_):
    out = []
    for logp in range(1, 5):
        for lines in LINES:
            try:
                plan.set_tiles(pass_, logp, lines)
            except mwntt.MwError:
                continue
            out.append((logp, lines))
    return out


def _splits(log2n, limbs):
    max_full = {1: 13, 2: 12, 4: 11}[limbs]
    s = [0] if log2n <= max_full else []
    s += [l1 for l1 in range(3, 10) if 3 <= log2n - l1 <= 9]
    return s


def _time(plan, x, y, z, batch, reps):
    import torch
    for _ in range(2):
        plan.forward(y, x, batch=batch)
        plan.inverse(z, y, batch=batch)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        plan.forward(y, x, batch=batch)
        plan.inverse(z, y, batch=batch)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e3 / reps / batch / 2     # us per transform


def tune(log2n: int, bits: int, batch: int, reps: int = 10, seed: int = 7) -> dict:
    import torch
    q = W.find_prime(bits, seed)
    limbs = W.limbs_for_bits(bits)
    n = 1 << log2n
    plan = mwntt.ntt_plan(log2n, q, limbs)
    x = mwntt.to_device(W.uniform_residues(W.rng(seed), q, n * batch, limbs))
    y, z = torch.empty_like(x), torch.empty_like(x)
    ref = None
    results = []

    def run(cfg):
        nonlocal ref
        apply(plan, cfg)
        us = _time(plan, x, y, z, batch, reps)
        if ref is None:
            ref = y.clone()
        if not torch.equal(y, ref) or not torch.equal(z, x):
            raise AssertionError(f"configuration {cfg} changed the result")
        results.append({"cfg": dict(cfg), "us_per_ntt": round(us, 4)})
        return us

    # bring clocks and code objects up before the first timing (otherwise the
    # first configuration measured reads slower than the same one measured later)
    import time
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < 0.05:
        plan.forward(y, x, batch=batch)
        plan.inverse(z, y, batch=batch)
    torch.cuda.synchronize()
    default = {"split": plan.split}
    if default["split"] == 0:
        default["full"] = plan.get_tiles(0)
    else:
        default["col"], default["row"] = plan.get_tiles(1), plan.get_tiles(2)
    default_us = run(default)
    for split in _splits(log2n, limbs):
        plan.split = split
        if split == 0:
            for shape in _valid_shapes(plan, 0):
                run({"split": 0, "full": shape})
            continue
        d_col, d_row = plan.get_tiles(1), plan.get_tiles(2)
        cols = _valid_shapes(plan, 1)
        plan.split = split
        rows = _valid_shapes(plan, 2)
        best_col, best_t = d_col, None
        for c in cols:
            t = run({"split": split, "col": c, "row": d_row})
            if best_t is None or t < best_t:
                best_col, best_t = c, t
        for r in rows:
            if r != d_row:
                run({"split": split, "col": best_col, "row": r})
    plan.destroy()
    results.sort(key=lambda r: r["us_per_ntt"])
    return {"log2n": log2n, "bits": bits, "batch": batch, "best": results[0],
            "default": {"cfg": default, "us_per_ntt": round(default_us, 4)},
            "candidates": len(results), "ranked": results[:12]}


def emit_header(jsonl_paths, out_path: str) -> None:
    """Write the tuned-configuration table (C header) from autotuner JSONL output.

    Batch 1 results become the latency entries, the largest batch per
    (width, N) the throughput entries."""
    best = {}
    for path in jsonl_paths:
        for line in open(path):
            r = json.loads(line)
            key = (W.limbs_for_bits(r["bits"]), r["log2n"])
            kind = 0 if r["batch"] == 1 else 1
            cur = best.get((key, kind))
            if kind == 1 and cur is not None and cur[0] > r["batch"]:
                continue
            best[(key, kind)] = (r["batch"], r["best"]["cfg"], r["best"]["us_per_ntt"])
    rows = []
    for ((limbs, log2n), kind), (batch, cfg, us) in sorted(best.items()):
        full = cfg.get("full", (0, 0))
        col = cfg.get("col", (0, 0))
        row = cfg.get("row", (0, 0))
        rows.append(f"    {{{limbs}, {log2n}, {kind}, {cfg['split']}, {full[0]}, {full[1]}, {col[0]}, {col[1]}, "
                    f"{row[0]}, {row[1]}}},  // batch {batch}: {us} us per transform")
    text = """// Tuned NTT decompositions and tile shapes for MI355X (gfx950).
// Generated by `python -m paper_2509_12494_amd.autotune ... --emit-header` from
// measured sweeps (forward + inverse round trips, every candidate checked bit
// for bit against the default configuration).  kind 0: latency (one
// transform per call), kind 1: throughput (large batches).
#pragma once
#include <stdint.h>

namespace mw {

struct TunedCfg {
  uint8_t limbs, log2n, kind, log_n1;
  uint8_t full_logp;
  uint16_t full_lines;
  uint8_t col_logp, col_lines, row_logp, row_lines;
};

static const TunedCfg kTuned[] = {
%s
};

}  // namespace mw
""" % "\n".join(rows)
    with open(out_path, "w") as f:
        f.write(text)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--emit-header", nargs=2, metavar=("JSONL", "HEADER"),
                    help="write the tuned table from a sweep's JSONL instead of sweeping")
    ap.add_argument("--log2n", type=int, nargs="+", default=[16])
    ap.add_argument("--bits", type=int, nargs="+", default=[124])
    ap.add_argument("--batch", type=int, nargs="+", default=[1, 64])
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    if args.emit_header:
        emit_header([args.emit_header[0]], args.emit_header[1])
        return 0
    out = open(args.out, "a") if args.out else None
    for bits in args.bits:
        for log2n in args.log2n:
            for batch in args.batch:
                r = tune(log2n, bits, batch, args.reps)
                line = json.dumps(r)
                print(json.dumps({k: r[k] for k in ("log2n", "bits", "batch", "best", "default", "candidates")}),
                      flush=True)
                if out:
                    out.write(line + "\n")
                    out.flush()
    if out:
        out.close()


if __name__ == "__main__":
    sys.exit(main())
