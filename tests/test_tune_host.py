"""Host logic of the launch-schedule autotuner (paper_1412_2480_amd/tune.py):
shapes whose LDS staging does not fit are skipped, shapes whose tile slots
overflow while being timed are skipped, any other library error is
raised, every context is closed, and within the 2% tie the earlier candidate
wins. A stand-in for the library context supplies the timings, so this runs
without a GPU; the GPU test of the tuner times real steps."""
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import paper_1412_2480_amd as pic  # noqa: E402
from paper_1412_2480_amd import tune  # noqa: E402


class FakeSim:
    """Times a step at ms_of(options) ms; raises where `fail` says so."""
    created = []
    ms_of = None
    fail = {}

    def __init__(self, runs, opts):
        self.opts = opts
        self.closed = False
        self.steps = 0
        FakeSim.created.append(self)

    def _key(self):
        return (self.opts.tile_x, self.opts.tile_y)

    def step(self, n=1):
        code = FakeSim.fail.get(self._key())
        if code is not None:
            raise pic.PicError(code, "stand-in failure")
        self.steps += n

    def tune(self, steps=3, splits=(), cg_blocks=()):
        return dict(tile_split=2, cg_blocks=128)

    def timing(self, on=True):
        self.steps = 0

    def get_timing(self):
        ms = FakeSim.ms_of(self.opts) * self.steps
        return {"push": dict(ms=0.8 * ms, launches=self.steps),
                "sort": dict(ms=0.2 * ms, launches=max(1, self.steps // 4)),
                "graph_replays": 0}

    def close(self):
        self.closed = True


def _no_fit(runs, opts):
    if (opts.tile_x, opts.tile_y) == (16, 32):
        raise pic.PicError(-1, "tile too large for LDS")


@pytest.fixture
def fake(monkeypatch):
    FakeSim.created = []
    FakeSim.fail = {}
    monkeypatch.setattr(tune, "Sim", FakeSim)
    monkeypatch.setattr(tune, "plan", _no_fit)
    return FakeSim


def test_shape_search_skips_misfits_and_overflows_and_breaks_ties_early(fake):
    ms = {(4, 32): 2.00, (8, 32): 1.99, (16, 32): 1.0, (16, 16): 1.5, (8, 16): 2.5}
    fake.ms_of = lambda o: ms[(o.tile_x, o.tile_y)]
    fake.fail = {(16, 16): -5}          # a tile's slots overflow while timed
    best, table = tune.autotune([None], lambda sim: None, {"precision": "fp32"},
                                shapes=((4, 32), (8, 32), (16, 32), (16, 16), (8, 16)))
    assert [r["tile"] for r in table] == [(4, 32), (8, 32), (8, 16)]
    # (8, 32) is fastest, (4, 32) within 2% of it and earlier in the list
    assert best["tile"] == (4, 32)
    assert best["tile_split"] == 2 and best["cg_blocks"] == 128
    assert abs(table[1]["ms_per_step"] - 1.99) < 1e-12
    assert all(s.closed for s in fake.created)
    assert len(fake.created) == 4      # (16, 32) never got a context


def test_shape_search_outside_the_tie_takes_the_fastest(fake):
    ms = {(4, 32): 2.10, (8, 32): 2.00}
    fake.ms_of = lambda o: ms[(o.tile_x, o.tile_y)]
    best, _ = tune.autotune([None], lambda sim: None, {}, shapes=((4, 32), (8, 32)))
    assert best["tile"] == (8, 32)


def test_shape_search_raises_other_errors_and_closes(fake):
    fake.ms_of = lambda o: 1.0
    fake.fail = {(8, 32): -3}          # a HIP error is not a reason to skip
    with pytest.raises(pic.PicError) as e:
        tune.autotune([None], lambda sim: None, {}, shapes=((4, 32), (8, 32)))
    assert e.value.code == -3
    assert all(s.closed for s in fake.created)


def test_shape_search_with_nothing_left_fails_loudly(fake):
    fake.ms_of = lambda o: 1.0
    fake.fail = {(4, 32): -5}
    with pytest.raises(RuntimeError, match="no candidate"):
        tune.autotune([None], lambda sim: None, {}, shapes=((4, 32), (16, 32)))


@pytest.mark.parametrize("times,expect", [
    ({0: 2.90, 3: 2.60, 4: 2.58, 8: 2.70}, 3),   # 3 within 2% of the fastest, earlier
    ({0: 2.90, 3: 2.70, 4: 2.50, 8: 2.70}, 4),   # 3 outside the tie
    ({0: 2.50, 3: 2.44, 4: 2.40, 8: 2.60}, 3),   # 0 outside, 3 inside
])
def test_reordering_period_tie_rule(fake, times, expect):
    fake.ms_of = lambda o: times[o.sort_every]
    k, table = tune.tune_sort_every([None], lambda sim: None, {"tile": (4, 32)},
                                    candidates=(0, 3, 4, 8), steps=8, warmup=2)
    assert k == expect
    assert [r["sort_every"] for r in table] == [0, 3, 4, 8]
    for r in table:
        assert abs(r["ms_per_step"] - times[r["sort_every"]]) < 1e-12
    assert all(s.closed for s in fake.created)
