"""GPU tests of the autotuner: every launch choice it tries returns the same
results (it checks that itself), tuning never changes a search's results, the
tuned choice is what later searches of the same shape run, and the text cache
round-trips and loads only for a matching index."""
import os
import sys
import tempfile

import numpy as np
import pytest

from paper_2605_16007_amd import RbqError
from tests._parity import lib_index, make_case

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tcase():
    _say("[tune] mixture n=30000 d=128 nlist=64 nq=300")
    X, Q, idx = make_case(30_000, 128, 64, 300, seed=71)
    lib = lib_index(X, idx)
    yield X, Q, idx, lib
    lib.close()


@pytest.mark.parametrize("nprobe,R", [(4, 50), (32, 400)])
def test_autotune_keeps_results(tcase, nprobe, R):
    X, Q, idx, lib = tcase
    _say(f"[tune] nprobe={nprobe} R={R}")
    before = lib.search(Q, nprobe, 10, R)
    r = lib.autotune(Q, nprobe, 10, R)
    _say(f"[tune] chose {r}")
    # 361 launch choices, then four index-block sizes for a list-major winner
    assert r["scan"] in (1, 2) and r["chunk_group_min"] in (0, 4, 16, 64)
    assert r["trials"] == 361 + (4 if r["scan"] == 2 else 0) + 2
    assert r["merge_form"] in (0, 1, 2)
    assert r["block"] in (0, 8, 16, 32, 64) and (r["scan"] == 2 or r["block"] == 0)
    assert r["growth"] in (2, 3, 4, 6, 8)
    assert r["early_form"] in (0, 1)
    assert r["group_size"] in (32, 64) and r["wg_per_cu"] in (4, 8) and r["first_factor"] in (1, 2, 4)
    assert r["ms"] > 0 and r["ms"] <= r["ms_default"] * 1.5
    after = lib.search(Q, nprobe, 10, R)
    np.testing.assert_array_equal(before[0], after[0])
    np.testing.assert_array_equal(before[1], after[1])
    # the tuned scan form is the one that runs
    lib.set_timing(True)
    lib.search(Q, nprobe, 10, R)
    t = lib.timings()
    lib.set_timing(False)
    assert t["popc_launches"] + t["group_launches"] > 0
    if r["scan"] == 1:
        assert t["group_launches"] == 0
    elif r["chunk_group_min"] == 0:
        assert t["group_launches"] > 0 and t["popc_launches"] == 0


def test_tune_cache_round_trip(tcase):
    X, Q, idx, lib = tcase
    lib.autotune(Q[:100], 8, 10, 100)
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "tune.txt")
        lib.tune_save(path)
        lines = [l for l in open(path) if not l.startswith("#")]
        assert len(lines) >= 1 and "gfx950" in lines[0]
        other = lib_index(X, idx)  # same data and structure: same signature
        try:
            assert other.tune_load(path) == len(lines)
        finally:
            other.close()
        X2, _, idx2 = make_case(8_000, 128, 16, 4, seed=72)
        diff = lib_index(X2, idx2)  # another index: nothing loads
        try:
            assert diff.tune_load(path) == 0
            diff.tune_save(path)  # keeps the first index's lines
            assert len([l for l in open(path) if not l.startswith("#")]) == len(lines)
        finally:
            diff.close()
        with open(path, "a") as f:
            # signature, key, scan 7 (out of range), G, wg_per_cu, first_factor, gm, growth, early,
            # block, merge
            f.write(lines[0].rsplit(" ", 11)[0] + " 5 7 32 8 2 4 2 0 0 0\n")
        with pytest.raises(RbqError):
            lib.tune_load(path)
    lib.tune_clear()
