"""The persistent stages' hand-out of work items (the device's work_next /
work_end), replayed on the CPU with blocks interleaved at random: with and
without the next-item request, every item of an XCD's range is processed by
exactly one block, every block stops, and the counters are back at zero,
with no request after that reset, when the launch ends."""
import random

import pytest


def run_launch(ranges, blocks_per_xcd, prefetch, seed):
    rng = random.Random(seed)
    counters = [0] * 9                      # 8 per-XCD item counters + the finished-block count
    processed = []
    events = []                             # ("atomic", x) / ("reset",) in issue order
    blocks = []
    for x in range(8):
        for _ in range(blocks_per_xcd):
            blocks.append({"x": x, "next": -1, "state": "ask", "item": None})

    def atomic(x):
        events.append(("atomic", x))
        v = counters[x]
        counters[x] += 1
        return v

    live = list(range(len(blocks)))
    while live:
        bi = rng.choice(live)
        b = blocks[bi]
        x, (base, end) = b["x"], ranges[b["x"]]
        if b["state"] == "ask":             # work_next
            item = b["next"] if b["next"] >= 0 else base + atomic(x)
            if prefetch:
                b["next"] = base + atomic(x) if item < end else end
            if item < end:
                b["item"], b["state"] = item, "work"
            else:
                b["state"] = "end"
        elif b["state"] == "work":          # the item's work, then ask again
            processed.append((x, b["item"]))
            b["state"] = "ask"
        else:                               # work_end: the last block clears the counters
            counters[8] += 1
            if counters[8] == len(blocks):
                for k in range(9):
                    counters[k] = 0
                events.append(("reset",))
            live.remove(bi)
    return processed, counters, events


@pytest.mark.parametrize("prefetch", [False, True])
@pytest.mark.parametrize("seed", range(20))
def test_items_processed_once_and_counters_cleared(prefetch, seed):
    rng = random.Random(1000 + seed)
    cuts = sorted(rng.randint(0, 300) for _ in range(7))
    xb = [0] + cuts + [300 + rng.randint(0, 50)]
    ranges = [(xb[x], xb[x + 1]) for x in range(8)]
    processed, counters, events = run_launch(ranges, rng.randint(1, 6), prefetch, seed)
    want = sorted((x, i) for x in range(8) for i in range(*ranges[x]))
    assert sorted(processed) == want                 # each item exactly once, by its own XCD
    assert counters == [0] * 9                       # ready for the next launch (or graph replay)
    assert events[-1] == ("reset",)                  # no counter request after the reset
