"""Host-side logic that needs no GPU: the autotuner's cache key and cache file."""

import json

from paper_1311_4627_amd import autotune, hsd


class _FakeCtx:
    def __init__(self, bins, L=500):
        self.n_bins = dict(enumerate(bins))
        self.L = L


def test_batch_key_groups_bins_by_solver_class():
    ctx = _FakeCtx([1024, 128, 512, 256, 16, 544, 272])
    key = json.loads(autotune.batch_key(ctx, list(range(7)), 16384, "dev"))
    assert key["bins"] == [[544, 1024], [272, 512], [256], [16, 128]]
    assert key["L"] == 500 and key["n_cells"] == 16384 and key["device"] == "dev" and key["tuner"] == "plan"
    # the class table matches the ranges the header documents
    assert hsd.CLASS_BINS == ((513, 1024), (257, 512), (129, 256), (16, 128))


def test_batch_key_ignores_grain_order_and_depends_on_batch():
    ctx = _FakeCtx([1024, 128, 512])
    assert autotune.batch_key(ctx, [0, 1, 2], 10, "d") == autotune.batch_key(ctx, [2, 0, 1], 10, "d")
    assert autotune.batch_key(ctx, [0, 1, 2], 10, "d") != autotune.batch_key(ctx, [0, 1, 2], 11, "d")
    assert autotune.batch_key(ctx, [0, 1], 10, "d") != autotune.batch_key(ctx, [0, 1, 2], 10, "d")
