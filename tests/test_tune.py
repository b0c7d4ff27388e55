"""Autotuner host logic (no GPU): cache keys carry the device, the library
build and the batch class, a cache of another version is ignored, lookups return the stored
knobs, every candidate is a valid plan whose knobs round-trip through
sfft_plan_info, and out-of-range knob values are rejected."""
import json

import pytest

import paper_2011_05749_amd as sfft
from paper_2011_05749_amd import tune


def test_cache_roundtrip_and_version(tmp_path):
    path = str(tmp_path / "c.json")
    key = tune.shape_key(2 ** 20, 256, 4, 2, 512, 1, device="gfx950-256cu", lib="abc")
    assert "gfx950-256cu" in key and "abc" in key and "N=1048576" in key and "mode=1" in key
    json.dump({"version": tune.CACHE_VERSION, "entries": {key: {"best": {"l1_resolve": 0, "jump_L": 64}}}},
              open(path, "w"))
    got = tune.lookup(2 ** 20, 256, 4, 2, 512, "noisy", path=path, device="gfx950-256cu", lib="abc")
    assert got == {"l1_resolve": 0, "jump_L": 64}
    # default B0 (next pow2 >= 2K) resolves to the same key
    assert tune.lookup(2 ** 20, 256, 4, 2, 0, 1, path=path, device="gfx950-256cu", lib="abc") == got
    # another library build or device: not found
    assert tune.lookup(2 ** 20, 256, 4, 2, 512, 1, path=path, device="gfx950-256cu", lib="abd") == {}
    assert tune.lookup(2 ** 20, 256, 4, 2, 512, 1, path=path, device="gfx942-304cu", lib="abc") == {}
    # the batch class is part of the key: batches up to the next power of two share it
    kb = tune.shape_key(2 ** 20, 256, 4, 2, 512, 1, device="gfx950-256cu", lib="abc", batch=48)
    assert kb.endswith("|batch=64") and key.endswith("|batch=1")
    assert tune.batch_class(64) == 64 and tune.batch_class(65) == 128 and tune.batch_class(1) == 1
    json.dump({"version": tune.CACHE_VERSION, "entries": {kb: {"best": {"jump_L": 32, "l1_resolve": 0}}}},
              open(path, "w"))
    assert tune.lookup(2 ** 20, 256, 4, 2, 512, 1, path=path, device="gfx950-256cu", lib="abc",
                       batch=64) == {"jump_L": 32, "l1_resolve": 0}
    assert tune.lookup(2 ** 20, 256, 4, 2, 512, 1, path=path, device="gfx950-256cu", lib="abc", batch=33) != {}
    assert tune.lookup(2 ** 20, 256, 4, 2, 512, 1, path=path, device="gfx950-256cu", lib="abc") == {}
    # a cache written by another format version is ignored
    json.dump({"version": tune.CACHE_VERSION + 1, "entries": {key: {"best": {"jump_L": 0}}}}, open(path, "w"))
    assert tune.lookup(2 ** 20, 256, 4, 2, 512, 1, path=path, device="gfx950-256cu", lib="abc") == {}
    assert tune.lookup(1, 1, 1, 2, path=str(tmp_path / "missing.json"), device="d", lib="l") == {}


@pytest.mark.parametrize("N,K,R,D,B0", [(2 ** 20, 256, 4, 2, 512), (2 ** 22, 1024, 4, 2, 2048),
                                        (2 ** 14, 40, 2, 3, 64), (2 ** 24, 4096, 4, 2, 8192)])
def test_candidates_are_valid_plans(N, K, R, D, B0):
    eligible = bool(sfft.Plan(N, K, R, D, B0=B0).info.l1_resolve)
    cands = tune.candidates(N, B0, D, eligible)
    assert cands[0] == tune.default_knobs(B0, D, eligible)
    assert len({json.dumps(c, sort_keys=True) for c in cands}) == len(cands)
    for c in cands:
        p = sfft.Plan(N, K, R, D, B0=B0, **c)
        assert p.info.fft_tile_lg == c["fft_tile_lg"] and p.info.gather_unroll == c["gather_unroll"]
        assert p.info.l1_resolve == (c["l1_resolve"] if eligible else 0)
    d = sfft.Plan(N, K, R, D, B0=B0).info
    assert d.fft_tile_lg == cands[0]["fft_tile_lg"] and d.gather_unroll == 4


def test_knob_validation():
    top = sfft.Plan(2 ** 16, 64, 2, 2, B0=2048).info.fft_tile_lg
    assert top == 11
    assert sfft.Plan(2 ** 16, 64, 2, 3, B0=8192).info.fft_tile_lg == 11   # D = 3: 2^13 / 4
    for bad in (dict(fft_tile_lg=4), dict(fft_tile_lg=12), dict(gather_unroll=3), dict(gather_unroll=16)):
        with pytest.raises(sfft.SfftError):
            sfft.Plan(2 ** 16, 64, 2, 2, B0=2048, **bad)


def test_choose_keeps_the_default_within_the_margin():
    # medians with the default's first
    assert tune.choose([1.00, 0.99, 1.05], 0.02) == 0      # 1 % faster: noise, keep the default
    assert tune.choose([1.00, 0.97, 0.975], 0.02) == 1     # 3 % faster: taken
    assert tune.choose([1.00, 0.99, 0.95], 0.02) == 2      # the fastest, not the first past the margin
    assert tune.choose([1.00, 1.10], 0.02) == 0            # slower candidates never win
    assert tune.choose([1.00], 0.02) == 0
