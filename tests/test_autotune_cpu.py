"""The schedule autotuner's cache logic, on the CPU (the timing itself needs a GPU).

``tune`` times every candidate schedule of a size with ``time_schedule``; here that function is
replaced by a fixed table, so what is checked is the bookkeeping: the fastest candidate is
recorded with its split variant and stream groups, ``schedule_for`` returns it, entries marked
``pinned`` are kept, and sizes without split-x2 kernels get no split candidates.
"""
import json

import pytest

from paper_2211_10185_amd import autotune as A


def fake_times(table):
    def time_schedule(N, prec, k, sched, steps):
        return table[A.candidate_name(sched, N)]
    return time_schedule


def test_candidates_name_every_variant_and_grouping():
    names = [A.candidate_name(c, 160) for c in A.candidates(160, 0, 3)]
    assert names == ["rowcol/1stream", "split/4col", "split/4col/2streams", "split/4col/3streams",
                     "split/2col", "split/2col/2streams", "split/2col/3streams", "split-swapped",
                     "split-swapped/2streams", "split-swapped/3streams"]
    # 250: 4 does not divide N (no separate 2-column variant); 256: the 8-row variant, no swapped one
    assert [A.candidate_name(c, 250) for c in A.candidates(250, 0, 1)] == ["rowcol/1stream", "split/2col",
                                                                          "split-swapped"]
    assert "split8row/8col" in [A.candidate_name(c, 256) for c in A.candidates(256, 0, 1)]
    assert "split-swapped" not in [A.candidate_name(c, 256) for c in A.candidates(256, 0, 1)]
    # complex128 and sizes without split-x2 kernels: no split candidate
    assert not any(c["split"] for c in A.candidates(256, 1, 3))
    assert not any(c["split"] for c in A.candidates(64, 0, 3))


def test_tune_records_the_fastest_and_keeps_pinned_entries(tmp_path, monkeypatch):
    path = tmp_path / "tuning.json"
    pinned = {"rowcol": True, "single_stream": True, "groups": 1, "split": False, "pinned": "chosen elsewhere"}
    path.write_text(json.dumps({"entries": {"160/0/1": pinned}}))
    table = {n: 100.0 for n in [A.candidate_name(c, 160) for c in A.candidates(160, 0, 3)]}
    table["split-swapped/2streams"] = 50.0
    monkeypatch.setattr(A, "time_schedule", fake_times(table))
    monkeypatch.setattr(A, "_device_name", lambda: "test")
    monkeypatch.setenv("QFDTD_TUNING", str(path))
    A._cache = None
    A.tune([160], precisions=(0,), states=(1, 3), path=str(path), verbose=False)
    doc = json.loads(path.read_text())
    assert doc["entries"]["160/0/1"] == pinned
    e = doc["entries"]["160/0/2"]
    assert e["split"] and e["split_variant"] == 3 and e["groups"] == 2 and not e["single_stream"]
    assert A.schedule_for(160, 2, 0, 3) == {"rowcol": False, "single_stream": False, "groups": 2, "split": True,
                                            "split_variant": 3}
    assert A.schedule_for(160, 2, 0, 1)["rowcol"] is True
    # FDTD never uses an FFT schedule
    assert A.schedule_for(160, 0, 0, 3)["split"] is False
    A._cache = None


def test_shipped_cache_pins_are_explained():
    doc = json.load(open(A.os.path.join(A.HERE, "tuning.json")))
    for k, e in doc["entries"].items():
        if "pinned" in e:
            assert isinstance(e["pinned"], str) and len(e["pinned"]) > 40, k
