"""Host logic of the tuning search (no GPU): coordinate descent over the knobs, invalid
candidates skipped, the JSON cache written, keyed and read back."""
from __future__ import annotations

import json

import pytest

import paper_1501_04784_amd as kb
from paper_1501_04784_amd import autotune


@pytest.fixture
def fake_device(monkeypatch):
    monkeypatch.setattr(autotune, "arch", lambda: "gfx950")
    monkeypatch.setattr(autotune.torch.cuda, "empty_cache", lambda: None)
    # a "build" returns its modelled time instead of running
    monkeypatch.setattr(autotune, "time_ms", lambda run, reps=3, warmup=1: run())


def model(t: kb.Tuning) -> float:
    """A made-up cost with its minimum at block 128, bucket 14, sub 4, segment 8192;
    sub-bucket width 5 with bucket 16 is 'invalid'."""
    if t.sub_bits == 5 and t.bucket_bits == 16:
        raise kb.KBuildError("invalid for this shape")
    return (1.0 + (t.block != 128) + 0.5 * (t.bucket_bits != 14) + 0.25 * (t.sub_bits != 4)
            + 0.125 * (t.seg_pairs != 8192))


def test_search_reaches_the_modelled_optimum(fake_device):
    best, timings = autotune.search(lambda t: (lambda: model(t)), 8, "fp32fb64")
    assert best == kb.Tuning(block=128, bucket_bits=14, sub_bits=4, seg_pairs=8192)
    assert timings[best] == 1.0
    assert all(v != float("inf") for v in timings.values())


def test_tiles_follow_the_kernel_instantiations():
    assert autotune.axes(8, "fp64")["block"] == (0, 256, 192, 128)
    assert autotune.axes(8, "fp32fb64")["block"] == (0, 256, 128)
    assert autotune.axes(4, "fp64")["block"] == (0, 768, 384)
    assert autotune.axes(4, "fp32")["block"] == (0, 1024, 512)


def test_every_candidate_plans_or_is_refused_cleanly():
    """Each knob value alone is accepted by kb_plan for a brick batch of this size, or
    refused with an argument error (never a crash)."""
    for elem in (4, 8):
        for prec in ("fp32fb64", "fp64"):
            for knob, values in autotune.axes(elem, prec).items():
                for v in values:
                    try:
                        kb.plan(elem, 50_000, 60_000, prec, autotune._with(kb.Tuning(), knob, v))
                    except kb.KBuildError as e:
                        assert "invalid argument" in str(e)


def test_cache_round_trip(fake_device, tmp_path):
    path = str(tmp_path / "sub" / "tuning.json")
    calls = []

    def make_run(t):
        calls.append(t)
        return lambda: model(t)

    t1, e1 = autotune.tuned("batch", 8, "fp32fb64", 36 * 11_600_617, make_run, cache_path=path)
    assert e1["source"] == "search" and e1["ms"] == 1.0 and e1["default_ms"] == model(kb.Tuning())
    n = len(calls)
    t2, e2 = autotune.tuned("batch", 8, "fp32fb64", 36 * 11_600_617, make_run, cache_path=path)
    assert e2["source"] == "cache" and t2 == t1 and len(calls) == n  # nothing timed
    data = json.load(open(path))
    assert list(data) == ["gfx950/batch/8/2/29"]  # arch / kind / element / precision / log2 pairs
    # another size class, precision or kind searches again
    autotune.tuned("batch", 8, "fp64", 36 * 11_600_617, make_run, cache_path=path)
    autotune.tuned("batch", 8, "fp32fb64", 36 * 1_000, make_run, cache_path=path)
    assert len(json.load(open(path))) == 3
    t3, e3 = autotune.tuned("batch", 8, "fp32fb64", 36 * 11_600_617, make_run, cache_path=path, refresh=True)
    assert e3["source"] == "search" and t3 == t1


def test_joint_coordinate_finds_a_pair_that_neither_knob_finds_alone(fake_device):
    """Sub-bucket width 5 pays only with 1024 table slots (each alone is slower than the
    built-in choice): one coordinate over both reaches the pair."""
    def cost(t: kb.Tuning) -> float:
        if (t.sub_bits, t.table_slots) == (5, 1024):
            return 0.5
        return 1.0 + 0.5 * (t.sub_bits == 5) + 0.25 * (t.table_slots != 0)

    best, _ = autotune.search(lambda t: (lambda: cost(t)), 8, "fp64")
    assert (best.sub_bits, best.table_slots) == (5, 1024)
