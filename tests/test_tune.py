"""Autotuner host logic (CPU): buckets, batch keys, cache round trip."""
import dataclasses
import json

import synth
from paper_1803_07772_amd import Params, tune


def test_bucket_rounds_up_to_powers_of_two():
    assert tune.bucket(5, 64, 32, 2) == "M8-N64-K32-l2"
    assert tune.bucket(17, 1024, 256, 3) == "M32-N1024-K256-l3"
    assert tune.bucket(1, 1, 1, 1) == "M1-N1-K1-l1"


def test_batch_key_is_the_median_work_drop():
    small = [synth.make_drop(synth.CFG2, s, 0) for s in range(5)]
    big = synth.make_drop(synth.CFG2.with_sizes(9, 512, 100), 0, 0)
    # one big drop outweighs five small ones
    assert tune.batch_key(small + [big]) == tune.bucket(9, 512, 100, big.l)
    assert tune.batch_key(small) == "M8-N64-K32-l2"


def test_tuned_params_from_cache(tmp_path):
    drops = [synth.make_drop(synth.CFG2, s, 0) for s in range(3)]
    cache = {"M8-N64-K32-l2": {"lds_kb": 79, "tile": 8}}
    p = tune.tuned(drops, Params(fixed_count=0), cache)
    assert p == dataclasses.replace(Params(fixed_count=0), lds_kb=79, tile=8)
    assert tune.tuned(drops, Params(), {}) == Params()
    full = {"M8-N64-K32-l2": {"lds_kb": 0, "tile": 0, "block": 256, "wave": 2}}
    assert tune.tuned(drops, Params(), full) == dataclasses.replace(Params(), block=256, wave=2)
    path = tmp_path / "c.json"
    tune.save_cache(cache, str(path))
    assert tune.load_cache(str(path)) == cache
    assert json.loads(path.read_text()) == cache


def test_schedule_from_cache_and_group_candidates():
    drops = [synth.make_drop(synth.CFG2, s, 0) for s in range(3)]
    cache = {"M8-N64-K32-l2": {"lds_kb": 0, "tile": 0, "block": 1024, "wave": 0, "group_triples": 4000}}
    assert tune.tuned(drops, Params(), cache) == dataclasses.replace(Params(), block=1024, group_triples=4000)
    big = synth.make_drop(synth.CFG2.with_sizes(9, 512, 100), 0, 0)
    g = tune.group_candidates(drops + [big])
    assert g[0] == 0 and g[1:] == [9 * 512 * 100 // 2, 9 * 512 * 100 // 4, 9 * 512 * 100 // 8]
