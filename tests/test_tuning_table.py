"""The packaged tile table (tuned_mi355x.json) on the CPU: every entry is
keyed in the current format, names a configuration the tuner would have
timed for that stencil and grid, and records the fastest of its own timings,
so that a hand edit or a stale entry cannot pass for a tuned one."""
import json

import pytest

pytest.importorskip("torch")

from paper_2606_04882_amd import autotune as A  # noqa: E402


def entries():
    with open(A.PACKAGED) as f:
        return json.load(f)


def test_keys_are_current():
    for key in entries():
        assert key.startswith("v5|gfx950-"), key


def test_single_shot_entries_are_tuned_choices():
    n = 0
    for key, e in entries().items():
        parts = key.split("|")
        if parts[2] == "batched":
            continue
        ndim, shape, M = int(parts[2]), parts[3], int(parts[4])
        grid = [int(x) for x in parts[5].split("x")]
        cands = A.candidates(ndim, shape, M, grid[0] if ndim == 3 else 0)
        pick = (e["rows"], e["zchunk"], e.get("tsteps", 1))
        assert pick in cands, (key, pick)
        label = f"{pick[0]}x{pick[1]}x{pick[2]}"
        assert set(e["ms"]) <= {f"{r}x{z}x{t}" for r, z, t in cands}, key
        assert min(e["ms"], key=e["ms"].get) == label, (key, label)
        n += 1
    assert n >= 8


def test_batched_entries():
    n = 0
    for key, e in entries().items():
        if key.split("|")[2] != "batched":
            continue
        names = key.split("|")[4].split(",")
        assert sorted(e["rows"]) == sorted(names)
        for name, rows in e["rows"].items():
            assert rows in (4, 8), (name, rows)
            if "-cross-" in name:
                assert rows == 4, name     # crosses have one batched tile
        n += 1
    assert n >= 1
