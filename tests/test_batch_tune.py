"""The batch pass-shape table (paper_1502_05366_amd/batch_tuning.json, written
by the autotuner on a GPU) and its lookup, on the CPU."""

import json

import numpy as np

from paper_1502_05366_amd import batch_tune as BT


def test_size_classes_and_buckets():
    assert list(BT.size_class([1, 256, 257, 1024, 1025, 10 ** 6])) == [0, 0, 1, 1, 2, 2]
    table = {BT.bucket_key(0, 2, 32): 2, BT.bucket_key(2, 0, 80): 1}
    got = BT.choose([100, 3000, 100, 10], [4000, 200, 4000, 10], [17, 65, 16, 5], table=table)
    # (0, 2, lp 32) -> 2; (2, 0, lp 80) -> 1; (0, 2, lp 16) missing -> 0; tiny -> 0
    assert list(got) == [2, 1, 0, 0]
    # out-of-range entries fall back to shape 0
    assert list(BT.choose([100], [100], [16], table={BT.bucket_key(0, 0, 16): 7})) == [0]


def test_committed_table_is_complete_and_valid():
    with open(BT.TABLE_PATH) as f:
        data = json.load(f)
    keys = {BT.bucket_key(mc, nc, lp) for mc in range(3) for nc in range(3) for lp in BT.LPS}
    assert set(data["table"]) == keys
    assert all(0 <= v < BT.SHAPES for v in data["table"].values())
    # each entry is the fastest of its measured shapes
    for k, v in data["table"].items():
        ts = data["ms_per_batch"][k]
        assert len(ts) == BT.SHAPES and ts[v] == min(ts)
    assert BT.load_table() == {k: int(v) for k, v in data["table"].items()}
    ms, ns = np.array([64, 500, 2048]), np.array([2048, 64, 500])
    assert BT.choose(ms, ns, np.array([80, 9, 40])).dtype == np.int32
