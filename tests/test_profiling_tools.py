"""Host logic of the profiling helpers (paper_1805_06688_amd/profiling.py) on synthetic counter files."""
import csv
import json

import pytest

from paper_1805_06688_amd import profiling


def _counter_csv(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, value in rows:
            w.writerow({"Kernel_Name": name, "Grid_Size": "1024", "Counter_Name": counter, "Counter_Value": value})


# two launches of a class whose launch runs kernel A twice and kernel B once, plus an unrelated kernel
DISPATCHES = [("kA<1>", 10.0), ("kB<2>", 40.0), ("kA<1>", 30.0), ("kC", 999.0),
              ("kA<1>", 20.0), ("kB<2>", 60.0), ("kA<1>", 40.0)]


def test_traffic_counts_launches_by_one_kernel(tmp_path, capsys):
    f, w = tmp_path / "fetch.csv", tmp_path / "write.csv"
    _counter_csv(f, "FETCH_SIZE", DISPATCHES)
    _counter_csv(w, "WRITE_SIZE", [(n, v / 2) for n, v in DISPATCHES])
    profiling.traffic(str(f), str(w), 5, ["kA", "kB"], 2.0, 1.0, launches_of="kB")
    d = json.loads(capsys.readouterr().out)
    # per launch: FETCH (10+30+20+40)/2 = 50 KiB of kA, 50 KiB of kB; WRITE half of that
    assert d["launches"] == 2
    assert d["fetch_kib_per_launch"] == [50.0, 50.0]
    assert d["write_kib_per_launch"] == [25.0, 25.0]
    assert d["bytes_per_launch"] == (2.0 * 100.0 + 1.0 * 50.0) * 1024.0
    assert d["source_hash"] == profiling.source_hash()


def test_traffic_requires_one_dispatch_per_kernel_without_launches_of(tmp_path):
    f, w = tmp_path / "fetch.csv", tmp_path / "write.csv"
    _counter_csv(f, "FETCH_SIZE", DISPATCHES)
    _counter_csv(w, "WRITE_SIZE", DISPATCHES)
    with pytest.raises(SystemExit):
        profiling.traffic(str(f), str(w), 5, ["kA", "kB"])
    profiling.traffic(str(f), str(w), 5, ["kB"])          # one dispatch of kB per launch: accepted
