"""Autotuner of the batched randomized SVD: which pass shape (rsvd.h,
rsvd_batch_set_variants) is fastest for a matrix, by (m, n, l) bucket.

Buckets: m and n each in three classes (<= 256, <= 1024, larger) and the
padded sample size lp = 16 ceil(l / 16) in {16, 32, 48, 64, 80}.  The table
batch_tuning.json beside this file maps "m<class>n<class>lp<lp>" to a shape
index; BatchPlan applies it (shape 0 where a bucket is missing or there is
no table).

Running this module on a GPU measures the table: for every bucket a batch of
COUNT matrices with sizes drawn inside the bucket (seeded, the batch
workload's spectrum exp(-j/8)) is timed with each shape forced on all of its
matrices, and the fastest shape is kept.  The shapes differ only in the
order of the FP32 sums, so the choice never changes what is computed beyond
that order.

    python -m paper_1502_05366_amd.tune_batch     (writes batch_tuning.json)
"""

import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE_PATH = os.path.join(HERE, "batch_tuning.json")
EDGES = (256, 1024)             # class c: size <= EDGES[c] (last class: larger)
LPS = (16, 32, 48, 64, 80)
SHAPES = 3                      # RSVD_BATCH_VARIANTS

_table = None


def size_class(x):
    x = np.asarray(x)
    return np.searchsorted(np.asarray(EDGES), x, side="left")


def bucket_key(mc, nc, lp):
    return "m%dn%dlp%d" % (int(mc), int(nc), int(lp))


def load_table(path=TABLE_PATH):
    """The bucket -> shape table, or {} when there is none."""
    global _table
    if _table is None or path != TABLE_PATH:
        try:
            with open(path) as f:
                data = json.load(f)
            table = {str(k): int(v) for k, v in data.get("table", {}).items()}
        except FileNotFoundError:
            table = {}
        if path != TABLE_PATH:
            return table
        _table = table
    return _table


def choose(ms, ns, ls, table=None):
    """Shape index per matrix (int32 array)."""
    table = load_table() if table is None else table
    ms, ns, ls = np.asarray(ms), np.asarray(ns), np.asarray(ls)
    lps = 16 * ((ls + 15) // 16)
    out = np.zeros(len(ms), dtype=np.int32)
    for i, (mc, nc, lp) in enumerate(zip(size_class(ms), size_class(ns), lps)):
        v = table.get(bucket_key(mc, nc, lp), 0)
        out[i] = v if 0 <= v < SHAPES else 0
    return out
