"""Autotuner bookkeeping (CPU): cache keys and the stored tuning table."""
import json

from paper_2310_14746_amd import tune


def test_keys_distinguish_pattern_and_batch():
    assert tune._key(19, "f32", (512, 512, 512)) == "gfx950/D3Q19/f32/512x512x512"
    assert tune._key(19, "f32", (512, 512, 512), "aa") == "gfx950/D3Q19/f32-aa/512x512x512"
    a = [dict(shape=(32, 32, 32)), dict(shape=(48, 48, 48))]
    b = [dict(shape=(48, 48, 48)), dict(shape=(32, 32, 32))]
    ka, kb = tune._batch_key("f32", a), tune._batch_key("f32", b)
    assert ka != kb and ka.startswith("gfx950/batch/D3Q19/f32/2items-143360cells-")
    assert tune._batch_key("f32", a) == ka
    assert tune.lookup(19, "f32", (3, 5, 7)) == 0
    assert tune.lookup_row_pad(19, "f32", (3, 5, 7)) == 0
    assert all(p % 256 == 0 for p in tune.ROW_PADS) and 0 in tune.ROW_PADS
    assert tune.lookup_batch([dict(shape=(3, 5, 7))]) is None


def test_stored_entries_are_launchable():
    cache = json.load(open(tune.CACHE))
    assert cache
    for key, ent in cache.items():
        if "/batch/" in key:
            assert ent["tile"] % 64 == 0 and 64 <= ent["tile"] <= 512, key
            assert ent["blocks_per_cu"] >= 1 and 1 <= ent["chunk"] <= 64, key
        else:
            cap = 256 if "-aa/" in key else 1024
            # 0: the library's default width (an entry that only carries a row pad)
            assert ent["block_x"] % 64 == 0 and 0 <= ent["block_x"] <= cap, key
            pad = ent.get("row_pad", 0)
            assert pad % 256 == 0 and 0 <= pad <= 1 << 24, key
