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


def test_shipped_table_is_complete_and_accepted():
    """The launch table that ships for MI355X covers every (mode, dim, n) the
    forward entry points take, once, for one device key, and the library
    accepts every entry (the variant exists for that dimension)."""
    import os
    path = os.path.join(os.path.dirname(tune.__file__), "tuning", "gfx950.json")
    with open(path) as f:
        table = json.load(f)
    keys = [k.split("|") for k in table]
    assert {"|".join(k[:2]) for k in keys} and len({"|".join(k[:2]) for k in keys}) == 1
    seen = {(k[2], int(k[3]), int(k[4])) for k in keys}
    assert seen == {(m, d, n) for m in tune.MODES for d in (2, 3) for n in range(1, 17)}
    assert len(seen) == len(table)
    before = {(m, d, n): kron.kron_get_launch(m, d, n)
              for m in tune.MODES.values() for d in (2, 3) for n in range(1, 17)}
    try:
        for k, e in table.items():
            _, _, mode, dim, n = k.split("|")
            kron.kron_set_launch(tune.MODES[mode], int(dim), int(n), int(e["blocks_per_cu"]), int(e["variant"]))
            assert kron.kron_get_launch(tune.MODES[mode], int(dim), int(n)) == (e["blocks_per_cu"], e["variant"])
    finally:
        for (m, d, n), (b, v) in before.items():
            kron.kron_set_launch(m, d, n, b, v)
