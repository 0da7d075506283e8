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


def test_row_pad_and_block_width_entries_merge(tmp_path, monkeypatch):
    """Tuning the row pad keeps the stored block width and tuning the block
    width keeps the stored pad; the lowest mean over repetitions wins (a
    synthetic timing replaces the GPU)."""
    import sys
    import types
    out = str(tmp_path / "tuning.json")
    monkeypatch.setattr(tune, "CACHE", out)

    def fake_time(hlbm, lattice, storage, shape, block_x, steps, warmup, pattern="ab", row_pad=0):
        # fastest at block_x 256 and row_pad 8448; one slow allocation of the
        # best pad must not outweigh its mean
        fake_time.calls += 1
        slow = 0.03 if (row_pad == 8448 and not fake_time.slowed) else 0.0
        if slow:
            fake_time.slowed = True
        return 1.0 + abs(block_x - 256) / 1000 + abs(row_pad - 8448) / 1e5 + slow
    fake_time.calls = 0
    fake_time.slowed = False
    monkeypatch.setattr(tune, "time_block", fake_time)
    fake_torch = types.SimpleNamespace(empty=lambda *a, **k: None, uint8=None,
                                       cuda=types.SimpleNamespace(empty_cache=lambda: None))
    monkeypatch.setitem(sys.modules, "torch", fake_torch)
    import paper_2310_14746_amd.hlbm as hlbm_mod
    monkeypatch.setattr(hlbm_mod, "load", lambda: None)
    shape = (512, 32, 16)
    ent = tune.tune(19, "f32", shape, reps=2, write=True, out=out)
    assert ent["block_x"] == 256
    assert tune.lookup(19, "f32", shape) == ent["block_x"]
    res = tune.tune_row_pad(19, "f32", shape, reps=3, write=True, out=out)
    assert res["row_pad"] == 8448 and tune.lookup_row_pad(19, "f32", shape) == 8448
    assert tune.lookup(19, "f32", shape) == ent["block_x"]         # kept
    tune.tune(19, "f32", shape, reps=1, write=True, out=out)
    assert tune.lookup_row_pad(19, "f32", shape) == 8448          # kept
    stored = json.load(open(out))[tune._key(19, "f32", shape)]
    assert set(stored["row_pad_candidates"]) == {str(p) for p in tune.ROW_PADS}
