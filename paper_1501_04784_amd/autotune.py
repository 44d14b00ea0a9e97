"""Tuning search for the build's launch shape, with a JSON cache.

The knobs are those of ``kb_tuning``: the pass-1 element tile (elements per workgroup,
hence elements per wavefront), the first-level bucket width and the sub-bucket width
of the two partition passes (the widths of the "radix" digits the pairs are split on),
the segment length of the sub-bucket partition (pairs per chunk of a bucket), and the
slots of the hash table that sums a sub-bucket (fewer slots per entry let wider
sub-buckets keep the same local memory; too few send sub-buckets to the overflow path).
Every candidate runs the same kernels on the same inputs, so any valid candidate
gives the same matrix bit for bit; the search only times them.

The search is coordinate descent from the built-in choice: each knob in turn is set to
each of its values with the others held, the fastest kept, for up to three sweeps.  The
sub-bucket width and the table size are one coordinate (every pair of their values):
a wider sub-bucket pays only with a table that still lets as many workgroups share a
compute unit, so neither moves alone.  Results are
cached per (device architecture, build kind, element, precision, size class), the size
class being log2 of the number of lower pairs rounded to an integer, in a JSON file
(``KBUILD_TUNE_CACHE``, else ``~/.cache/kbuild/tuning.json``).
"""
from __future__ import annotations

import json
import math
import os
from dataclasses import asdict

import torch

from . import KBuildError, Tuning, _prec
from ._lib import KB_FP64

# element tiles the pass-1 kernels are instantiated for (kb_tuning.block), per
# (nodes per element, FP64 values): the built-in choice is the first, or the one the
# mesh shape selects among them
TILES = {(4, False): (1024, 512), (4, True): (768, 384), (8, False): (256, 128), (8, True): (256, 192, 128)}
BUCKET_BITS = (0, 12, 14, 16)
SUB_BITS = (0, 3, 4, 5)
SEG_PAIRS = (0, 4096, 8192)
TABLE_SLOTS = (0, 512, 1024, 2048)


def axes(elem: int, prec) -> dict:
    """Values of each coordinate of the search (0 = the library's own choice from the
    mesh shape); a coordinate named by a tuple of knobs takes tuples of their values."""
    return {"block": (0,) + TILES[(int(elem), _prec(prec) == KB_FP64)], "bucket_bits": BUCKET_BITS,
            ("sub_bits", "table_slots"): tuple((s, t) for s in SUB_BITS for t in TABLE_SLOTS),
            "seg_pairs": SEG_PAIRS}


def _with(t: Tuning, knob, value) -> Tuning:
    fields = dict(zip(knob, value)) if isinstance(knob, tuple) else {knob: value}
    return Tuning(**{**asdict(t), **fields})


def arch() -> str:
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def size_class(n_pairs: int) -> int:
    return int(round(math.log2(max(int(n_pairs), 1))))


def cache_key(kind: str, elem: int, prec, n_pairs: int) -> str:
    return f"{arch()}/{kind}/{int(elem)}/{_prec(prec)}/{size_class(n_pairs)}"


def default_cache_path() -> str:
    return os.environ.get("KBUILD_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "kbuild",
                                                               "tuning.json")


def load_cache(path: str | None = None) -> dict:
    path = path or default_cache_path()
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def store(key: str, entry: dict, path: str | None = None) -> None:
    path = path or default_cache_path()
    data = load_cache(path)
    data[key] = entry
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_ms(run, reps: int = 3, warmup: int = 1) -> float:
    """Mean time of ``run()`` (enqueues one build on the current stream), HIP events."""
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        run()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        run()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def search(make_run, elem: int, prec, reps: int = 3, warmup: int = 1, sweeps: int = 3):
    """Coordinate descent over ``axes``.  ``make_run(tuning)`` returns a callable that
    enqueues one build with that tuning, or raises KBuildError (or ValueError) when the
    tuning is not valid for the shape.  Returns (best Tuning, {Tuning: ms})."""
    timings: dict = {}

    def cost(t: Tuning) -> float:
        if t not in timings:
            try:
                timings[t] = time_ms(make_run(t), reps, warmup)
            except (KBuildError, ValueError):
                timings[t] = math.inf
            torch.cuda.empty_cache()  # the candidate's buffers go before the next one's
        return timings[t]

    best = Tuning()
    if cost(best) == math.inf:
        raise KBuildError("the built-in tuning is not valid for this shape")
    for _ in range(sweeps):
        moved = False
        for knob, values in axes(elem, prec).items():
            for v in values:
                t = _with(best, knob, v)
                if cost(t) < cost(best):
                    best, moved = t, True
        if not moved:
            break
    return best, {t: ms for t, ms in timings.items() if ms != math.inf}


def tuned(kind: str, elem: int, prec, n_pairs: int, make_run, cache_path: str | None = None, refresh: bool = False,
          reps: int = 3, warmup: int = 1):
    """The cached tuning for this (architecture, kind, element, precision, size class),
    searched and stored when absent (or when ``refresh``).  Returns (Tuning, entry) where
    entry holds the tuning, its time, the built-in choice's time and whether it came from
    the cache."""
    key = cache_key(kind, elem, prec, n_pairs)
    if not refresh:
        hit = load_cache(cache_path).get(key)
        if hit:
            try:
                return Tuning(**hit["tuning"]), {**hit, "source": "cache", "key": key}
            except (TypeError, KeyError):
                pass  # an entry from an older layout: search again
    best, timings = search(make_run, elem, prec, reps, warmup)
    entry = {"tuning": asdict(best), "ms": timings[best], "default_ms": timings.get(Tuning()),
             "candidates_timed": len(timings)}
    store(key, entry, cache_path)
    return best, {**entry, "source": "search", "key": key}
