"""Launch-shape table and its JSON persistence (host side, no GPU)."""
import json

import pytest

import paper_1304_7054_amd as kron
from paper_1304_7054_amd import tune


def test_set_get_and_reset():
    kron.kron_set_launch(kron.MODE_F32, 3, 7, -1, 0)   # the built-in default (a loaded table may differ)
    old = kron.kron_get_launch(kron.MODE_F32, 3, 7)
    kron.kron_set_launch(kron.MODE_F32, 3, 7, 2, 5)
    assert kron.kron_get_launch(kron.MODE_F32, 3, 7) == (2, 5)
    kron.kron_set_launch(kron.MODE_F32, 3, 7, -1, 0)
    assert kron.kron_get_launch(kron.MODE_F32, 3, 7) == old
    for bad in ((5, 3, 7, 0, 0), (-1, 3, 7, 0, 0), (0, 4, 7, 0, 0), (0, 3, 17, 0, 0), (0, 3, 7, 65, 0), (0, 3, 7, 0, 12), (0, 2, 7, 0, 5)):
        with pytest.raises(kron.KronError):
            kron.kron_set_launch(*bad)


def test_json_round_trip_applies_only_this_device(tmp_path, monkeypatch):
    monkeypatch.setattr(tune, "device_key", lambda: "gfx950|hip-test")
    table = {
        tune.entry_key("gfx950|hip-test", "f32", 2, 9): {"blocks_per_cu": 3, "variant": 1, "ms": 0.1},
        tune.entry_key("gfx942|hip-test", "f32", 2, 10): {"blocks_per_cu": 1, "variant": 2, "ms": 0.1},
    }
    path = tmp_path / "t.json"
    tune.save(table, str(path))
    assert json.loads(path.read_text()) == table
    before = kron.kron_get_launch(kron.MODE_F32, 2, 10)
    try:
        assert tune.load(str(path)) == 1
        assert kron.kron_get_launch(kron.MODE_F32, 2, 9) == (3, 1)
        assert kron.kron_get_launch(kron.MODE_F32, 2, 10) == before
    finally:
        kron.kron_set_launch(kron.MODE_F32, 2, 9, -1, 0)
