"""Host logic of the autotuner: cache keys, JSON round trip, re-application."""

import json

from paper_2005_09534_amd import autotune


class _FakeCtx:
    def __init__(self):
        self.calls = []

    def set_step_shape(self, L, nvec, precision, threads, lpl, wg_per_cu, lds_tables=1, early_loads=0,
                       rank_incremental=0, xcd_slices=1):
        self.calls.append(("shape", L, nvec, precision, threads, lpl, wg_per_cu, lds_tables,
                           early_loads, rank_incremental, xcd_slices))

    def set_block_size(self, L, precision, nev, block_size):
        self.calls.append(("block", L, precision, nev, block_size))


def test_shape_candidates_are_valid():
    assert len(autotune.SHAPES) == len(set(autotune.SHAPES))
    for t, lpl, wpc, lds, early, ranki, xcd in autotune.SHAPES:
        assert t in (256, 512, 1024) and lpl in (1, 2, 4) and lds in (0, 1) and early in (0, 1)
        assert ranki in (0, 1, 2) and wpc >= 1 and xcd in (1, 2, 4, 8)
        assert not (ranki == 2 and lds == 1)
    assert {sh[5] for sh in autotune.SHAPES} == {0, 1, 2}
    assert {sh[6] for sh in autotune.SHAPES} == {1, 2, 4, 8}


def test_staged_candidates_split_the_width():
    best = (256, 2, 8, 1, 0, 1, 1)
    for width in (1, 2, 4, 64):
        c = autotune.staged_candidates(best, width)
        assert all(sh[3:6] == best[3:6] and 2 <= sh[6] <= width for sh in c)
        assert {sh[6] for sh in c} == {x for x in (2, 4, 8) if x <= width}
        assert len(c) == len(set(c))


def test_cache_round_trip_and_apply(tmp_path):
    # older entries: six fields (no column slices), five (no rank mode)
    cache = {autotune._key("shape", 18, 0.0, 1, 32): [1024, 2, 2, 1, 0, 1, 2500.0],
             autotune._key("block", 18, 0.0, 1, 20): [8, 0.5],
             autotune._key("shape", 22, 1.0, 0, 16): [256, 1, 4, 0, 1, 1800.0],
             autotune._key("shape", 26, 0.0, 1, 64): [1024, 2, 2, 1, 0, 0, 8, 4000.0]}
    path = tmp_path / "tune.json"
    autotune.save_cache(cache, str(path))
    assert json.loads(path.read_text()) == cache
    back = autotune.load_cache(str(path))
    assert back == cache
    ctx = _FakeCtx()
    autotune.apply_cache(ctx, back)
    assert sorted(ctx.calls) == sorted([("shape", 18, 32, 1, 1024, 2, 2, 1, 0, 1, 1),
                                        ("block", 18, 1, 20, 8),
                                        ("shape", 22, 16, 0, 256, 1, 4, 0, 1, 0, 1),
                                        ("shape", 26, 64, 1, 1024, 2, 2, 1, 0, 0, 8)])


def test_missing_cache_is_empty(tmp_path):
    assert autotune.load_cache(str(tmp_path / "absent.json")) == {}


def test_cache_path_env(monkeypatch, tmp_path):
    monkeypatch.setenv("POLFED_TUNE_CACHE", str(tmp_path / "x.json"))
    assert autotune.cache_path() == str(tmp_path / "x.json")
