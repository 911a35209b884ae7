"""Host logic of the tile cache (paper_2607_07687_amd/autotune.py), with the
library calls replaced by recording fakes: the first call tunes and writes
the cache, later calls apply the cached sweep and two-sweep-pass choices,
entries without a pass choice are tuned again, and a handle that cannot run
passes gets separate sweeps instead of an error."""
import json

import pytest

from paper_2607_07687_amd import autotune as AT
from paper_2607_07687_amd import gmg as G

SHAPES = [(64, 32, 16), (32, 16, 8), (16, 8, 4)]


class Fake:
    def __init__(self, pair_ok=True):
        self.calls = []
        self.pair_ok = pair_ok

    def install(self, monkeypatch):
        monkeypatch.setattr(AT, "_arch", lambda: "gfx950")
        monkeypatch.setattr(G, "gmg_num_levels", lambda h: len(SHAPES))
        monkeypatch.setattr(G, "gmg_level_shape", lambda h, l: (SHAPES[l], (2, 2, 2)))
        monkeypatch.setattr(G, "gmg_autotune", self.autotune)
        monkeypatch.setattr(G, "gmg_set_tiles", self.set_tiles)
        monkeypatch.setattr(G, "gmg_set_pair_sweeps", self.set_pair)

    def autotune(self, h, x, sigma, reps):
        self.calls.append(("autotune", reps))
        return [dict(level=l, n=n, ty=8 if l == 0 else 1, kchunk=16 >> l, us=10.0 / (l + 1),
                     ty_default=8, kchunk_default=8, us_default=12.0,
                     pair_kchunk=(128 >> l) if l < 2 else 0, pair_ty=16 if l == 0 else 8,
                     us_pair=15.0)
                for l, n in enumerate(SHAPES)]

    def set_tiles(self, h, level, ty, kchunk):
        self.calls.append(("tiles", level, ty, kchunk))

    def set_pair(self, h, level, kchunk, ty=16):
        if kchunk and not self.pair_ok:
            raise G.GMGError(G.GMG_EINVAL, "no passes")
        self.calls.append(("pair", level, kchunk, ty if kchunk else None))


def test_tune_then_apply_cached_choices(tmp_path, monkeypatch):
    cache = str(tmp_path / "sub" / "tiles.json")
    f = Fake()
    f.install(monkeypatch)
    res = AT.tune(None, None, None, cache=cache, reps=3)
    assert f.calls == [("autotune", 3)]
    assert [r["pair_kchunk"] for r in res] == [128, 64, 0]
    table = json.load(open(cache))
    assert len(table) == 3
    key = "gfx950|64x32x16|f32|f32"
    assert table[key]["pair_kchunk"] == 128 and table[key]["ty"] == 8
    assert table[key]["pair_ty"] == 16
    f.calls.clear()
    res2 = AT.tune(None, None, None, cache=cache)
    assert ("autotune", 5) not in f.calls
    assert [c for c in f.calls if c[0] == "tiles"] == [("tiles", 0, 8, 16), ("tiles", 1, 1, 8),
                                                        ("tiles", 2, 1, 4)]
    assert [c for c in f.calls if c[0] == "pair"] == [("pair", 0, 128, 16), ("pair", 1, 64, 8),
                                                       ("pair", 2, 0, None)]
    assert all(r["cached"] for r in res2)


def test_entries_without_pass_choice_are_tuned_again(tmp_path, monkeypatch):
    cache = str(tmp_path / "tiles.json")
    # entries of an older cache: no pass choice, or no pass tile height
    old = {f"gfx950|{n[0]}x{n[1]}x{n[2]}|f32|f32": dict(ty=8, kchunk=8, us=1.0) for n in SHAPES}
    old[f"gfx950|{SHAPES[0][0]}x{SHAPES[0][1]}x{SHAPES[0][2]}|f32|f32"]["pair_kchunk"] = 64
    json.dump(old, open(cache, "w"))
    f = Fake()
    f.install(monkeypatch)
    AT.tune(None, None, None, cache=cache)
    assert f.calls[0][0] == "autotune"
    assert all("pair_kchunk" in v and "pair_ty" in v for v in json.load(open(cache)).values())


def test_cached_passes_fall_back_when_not_allowed(tmp_path, monkeypatch):
    cache = str(tmp_path / "tiles.json")
    Fake().install(monkeypatch)
    AT.tune(None, None, None, cache=cache)
    f = Fake(pair_ok=False)
    f.install(monkeypatch)
    AT.tune(None, None, None, cache=cache)
    assert [c for c in f.calls if c[0] == "pair"] == [("pair", 0, 0, None), ("pair", 1, 0, None),
                                                       ("pair", 2, 0, None)]


def test_no_cache_file_still_tunes(monkeypatch):
    f = Fake()
    f.install(monkeypatch)
    res = AT.tune(None, None, None, cache=None)
    assert f.calls == [("autotune", 5)] and len(res) == 3


@pytest.mark.parametrize("kind", ["f32", "bf16"])
def test_key_names_precision(kind):
    assert AT._key("gfx950", (8, 4, 2), "f32", kind) == f"gfx950|8x4x2|f32|{kind}"
