"""The grouped batches' tile cache (host-only: no GPU needed): orders below 1024 always take
the 128-row tile; an order the cache does not hold takes the 256-row default; a cached choice
is read back per architecture; a damaged file is ignored rather than trusted."""
import json
import os

import pytest

from paper_2602_19090_amd import binding as rb


@pytest.fixture
def cache_file(tmp_path, monkeypatch):
    path = tmp_path / "tiles.json"
    monkeypatch.setenv("REFEIG_TUNE_CACHE", str(path))
    return path


def test_small_orders_take_the_128_tile(cache_file):
    assert rb.tile_cache_lookup("gfx950", 256) == (True, 128)
    assert rb.tile_cache_lookup("gfx950", 768) == (True, 128)


def test_missing_entry_is_the_default(cache_file):
    assert rb.tile_cache_lookup("gfx950", 1024) == (False, 256)


def test_cached_choices_per_architecture(cache_file):
    cache_file.write_text(json.dumps({"gfx950:1280": 128, "gfx950:2048": 256, "gfx942:1280": 256}))
    assert rb.tile_cache_lookup("gfx950", 1280) == (True, 128)
    assert rb.tile_cache_lookup("gfx950", 2048) == (True, 256)
    assert rb.tile_cache_lookup("gfx942", 1280) == (True, 256)
    assert rb.tile_cache_lookup("gfx950", 1536) == (False, 256)


def test_damaged_cache_is_ignored(cache_file):
    cache_file.write_text('{"gfx950:1280": 77, "gfx950:1536": 128, garbage')
    assert rb.tile_cache_lookup("gfx950", 1280) == (False, 256)   # not a tile
    assert rb.tile_cache_lookup("gfx950", 1536) == (True, 128)


def test_bad_arguments():
    with pytest.raises(ValueError):
        rb.tile_cache_lookup("gfx950", 0)
