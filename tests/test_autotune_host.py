"""Host logic of the update autotuner, on the CPU: the coordinate descent
over the three shape knobs, with the GPU timing replaced by a cost surface
whose minimum is known."""

import pytest

torch = pytest.importorskip("torch")

from paper_1901_06207_amd import autotune  # noqa: E402


class _Stream:
    def __init__(self, n):
        self.shape = (n, 2)
        self.device = "cpu"


def _fake(monkeypatch, cost):
    calls = []

    def fake_time(cfg, streams, tuning, scratch, repeats, stream):
        calls.append(dict(tuning))
        return cost(tuning)

    monkeypatch.setattr(autotune, "_time", fake_time)
    monkeypatch.setattr(autotune.cbaa, "cbaa_update_batch_scratch_bytes",
                        lambda cfg, streams, t: 1 << 20)
    monkeypatch.setattr(autotune.cbaa, "scratch_tensor", lambda n, device="cuda": None)
    monkeypatch.setattr(autotune, "_key", lambda cfg, streams: None)
    return calls


def _streams():
    return [(_Stream(1000), _Stream(16), None, 0, 1)]


def test_separable_cost_finds_the_grid_minimum(monkeypatch):
    want = dict(chunk_pairs=65536, seg_records=16384, apply_blocks=768)

    def cost(t):
        return 1.0 + sum(abs(autotune_index(k, t[k]) - autotune_index(k, want[k]))
                         for k in want)

    calls = _fake(monkeypatch, cost)
    res = autotune.tune_update({}, _streams(), use_cache=False, stream=object())
    assert res["best"] == want
    assert res["best_ms"] == 1.0
    assert res["default_ms"] == cost(dict(chunk_pairs=16384, seg_records=65536,
                                          apply_blocks=512))
    # every timed shape is reported once, and the best is one of them
    keys = [tuple(sorted(c["tuning"].items())) for c in res["candidates"]]
    assert len(keys) == len(set(keys)) == len({tuple(sorted(c.items())) for c in calls})
    assert res["best"] in [c["tuning"] for c in res["candidates"]]


def test_coupled_cost_needs_the_second_sweep(monkeypatch):
    """A cost where the best segment size depends on the apply grid: the first
    sweep picks the segment while the grid is still the default, so only a
    second sweep reaches the joint minimum."""
    def cost(t):
        seg, blocks = t["seg_records"], t["apply_blocks"]
        if blocks == 2048:
            base = 4.0 if seg == 262144 else 7.0
        else:
            base = 8.0 if seg == 32768 else 10.0
        return base + (0.0 if t["chunk_pairs"] == 16384 else 0.5)

    _fake(monkeypatch, cost)
    one = autotune.tune_update({}, _streams(), use_cache=False, stream=object(), rounds=1)
    assert one["best"]["seg_records"] == 32768 and one["best"]["apply_blocks"] == 2048
    two = autotune.tune_update({}, _streams(), use_cache=False, stream=object(), rounds=2)
    assert two["best"] == dict(chunk_pairs=16384, seg_records=262144, apply_blocks=2048)
    assert two["best_ms"] == 4.0 < one["best_ms"]


def test_flat_cost_keeps_the_default_and_stops_after_one_sweep(monkeypatch):
    """Ties never move the shape (timing noise aside, a knob that does not
    matter keeps its default)."""
    calls = _fake(monkeypatch, lambda t: 2.0)
    res = autotune.tune_update({}, _streams(), use_cache=False, stream=object(), rounds=5)
    assert res["best"] == dict(chunk_pairs=16384, seg_records=65536, apply_blocks=512)
    # one sweep: the default plus the other four values of each knob
    assert len(calls) == 1 + 3 * 4


def autotune_index(knob, value):
    table = {"chunk_pairs": autotune.CHUNKS, "seg_records": autotune.SEGS,
             "apply_blocks": autotune.APPLY_BLOCKS}[knob]
    return table.index(value)
