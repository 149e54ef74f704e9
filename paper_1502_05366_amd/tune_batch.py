"""Measure the batch pass-shape table (batch_tune, batch_tuning.json) on the
current GPU: python -m paper_1502_05366_amd.tune_batch [--out PATH]."""

import argparse
import json
import sys
import time

import numpy as np

from . import batch_tune as BT

RANGES = ((64, 256), (257, 1024), (1025, 2048))   # sizes drawn per class
P, Q, SEED = 8, 1, 0x5EED0B07
REPS = 3


def bucket_batch(mc, nc, lp, count, g):
    ms = g.integers(RANGES[mc][0], RANGES[mc][1] + 1, count)
    ns = g.integers(RANGES[nc][0], RANGES[nc][1] + 1, count)
    # l = k + p inside (lp - 16, lp]
    lo = max(1, lp - 15 - P)
    ks = np.minimum(g.integers(lo, lp - P + 1, count), np.minimum(ms, ns)).astype(np.int32)
    return ms, ns, ks


def time_shape(R, torch, ms, ns, ks, buf, shape):
    plan = R.BatchPlan(ms, ns, ks, P, Q, variants=shape)
    out = plan.outputs()
    plan.run(buf, SEED, out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(REPS):
        plan.run(buf, SEED, out)
    e1.record()
    torch.cuda.synchronize()
    if int(out[3][0].item()) & (R.INFO_NONFINITE | R.INFO_BARRIER):
        raise RuntimeError("batch reported status %s" % out[3].cpu().numpy())
    return e0.elapsed_time(e1) / REPS


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--out", default=BT.TABLE_PATH)
    ap.add_argument("--count", type=int, default=256, help="matrices per bucket batch")
    args = ap.parse_args(argv)
    import torch
    import paper_1502_05366_amd as R
    from . import workloads as W

    if not torch.cuda.is_available():
        raise SystemExit("tune_batch needs a GPU")
    g = np.random.default_rng(SEED)
    table, times = {}, {}
    t0 = time.time()
    for mc in range(len(RANGES)):
        for nc in range(len(RANGES)):
            count = args.count // (2 if mc == 2 and nc == 2 else 1)
            for lp in BT.LPS:
                key = BT.bucket_key(mc, nc, lp)
                ms, ns, ks = bucket_batch(mc, nc, lp, count, g)
                As = W.c4_batch_torch(ms, ns, SEED + lp, "cuda")
                plan0 = R.BatchPlan(ms, ns, ks, P, Q, variants=0)
                buf = plan0.pack(As)
                del As, plan0
                ts = [time_shape(R, torch, ms, ns, ks, buf, v) for v in range(BT.SHAPES)]
                del buf
                torch.cuda.empty_cache()
                best = int(np.argmin(ts))
                table[key] = best
                times[key] = [round(t, 4) for t in ts]
                print("%-12s count %4d  ms per batch by shape %s -> %d (%.2fx of shape 0)"
                      % (key, count, times[key], best, ts[0] / ts[best]), flush=True)
    data = {
        "format": 1,
        "what": "fastest pass shape of the batched randomized SVD per (m, n, lp) bucket",
        "shapes": {"0": "128-row tiles, 64-deep chunks", "1": "256-row tiles, 32-deep chunks",
                   "2": "128-row tiles, 32-deep chunks"},
        "classes": {"0": "<= 256", "1": "257 .. 1024", "2": "> 1024"},
        "sampled_sizes": [list(r) for r in RANGES],
        "p": P, "q": Q, "count": args.count, "reps": REPS,
        "device": torch.cuda.get_device_name(0),
        "command": "python -m paper_1502_05366_amd.tune_batch",
        "table": table,
        "ms_per_batch": times,
    }
    with open(args.out, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
        f.write("\n")
    print("wrote %s in %.0f s" % (args.out, time.time() - t0), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
