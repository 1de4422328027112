"""Autotuner bookkeeping on the host: batch signatures and the JSON cache."""
import json

import numpy as np

import spgen
from paper_2106_14402_amd import autotune as AT


def _batch(n, seed):
    items = spgen.batch_mix(nprod=n, n_lo=256, n_hi=2048, config=3)
    return [it.A for it in items], [it.semiring for it in items]


def test_signature_is_stable_and_shape_sensitive():
    As, srs = _batch(6, 0)
    s1 = AT.signature(As, As, srs, "gfx950")
    s2 = AT.signature(As, As, srs, "gfx950")
    assert s1 == s2
    assert AT.signature(As, As, srs, "other") != s1                 # device is part of the key
    assert AT.signature(As[:3], As[:3], srs[:3], "gfx950") != s1    # so is the batch size and mix
    key = json.loads(s1)
    assert key["n"] == 6 and sum(c for _, c in key["mix"]) == 6


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    assert AT.load_cache(path) == {}
    AT.store_cache(path, {"k": {"knobs": {"short_seg": 8}, "ms": 1.0}})
    assert AT.load_cache(path)["k"]["knobs"]["short_seg"] == 8
    with open(path, "w") as f:
        f.write("not json")
    assert AT.load_cache(path) == {}


def test_candidates_start_from_defaults():
    for k, v in AT.BATCH_DEFAULTS.items():
        assert v in AT.CANDIDATES[k]
    assert set(AT.ORDER) == set(AT.CANDIDATES)
    o = AT.make_options(AT.BATCH_DEFAULTS)
    assert o.hash_max_nnz == 2048 and o.dense_threads == 512
