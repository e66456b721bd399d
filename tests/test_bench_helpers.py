"""The measurement plumbing of bench.py on the CPU: the committed counter
summaries are used only for their own workload, variant and kernel source
(a figure taken on other code reads as unmeasured), and the traffic is
the copy-calibrated sum of the raw counters."""
import json
import os

import pytest

import bench


def test_committed_counters_give_the_calibrated_traffic():
    for wl in ("clustered_512cubed_periodic", "lattice_64cubed_periodic"):
        rec = json.load(open(bench.counters_file(wl)))
        if rec["source_digest"] != bench.interact_source_digest():
            pytest.skip(f"{wl}: counters taken on other kernel source (profile again)")
        for key, v in rec["variants"].items():
            chunk, waves, pre = key.split("x")
            t = bench.interact_traffic(wl, int(chunk), int(waves), pre == "true")
            want = (v["fetch_kib_per_dispatch"] * rec["fetch_factor"] +
                    v["write_kib_per_dispatch"] * rec["write_factor"]) * 1024
            assert t is not None and abs(t["bytes_per_launch"] - want) <= 1e-6 * want, key
    e = bench.ewald_flops_per_particle("clustered_512cubed_periodic")
    assert e is not None and 5000 < e["flop_per_particle"] < 20000


def test_stale_or_foreign_counters_read_as_unmeasured(tmp_path, monkeypatch):
    assert bench.interact_traffic("clustered_512cubed_periodic", 99, 3, False) is None
    assert bench.interact_traffic("no_such_workload", 32, 3, False) is None
    # a summary taken on other kernel source
    src = bench.counters_file("clustered_512cubed_periodic")
    rec = json.load(open(src))
    rec["source_digest"] = "0" * 16
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / os.path.basename(src)).write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "counters_file", lambda wl: str(prof / os.path.basename(src)))
    assert bench.interact_traffic("clustered_512cubed_periodic", 32, 3, False) is None


def test_more_than_one_gpu_is_refused(monkeypatch, capsys):
    # one GPU only: the run ends with a message and status 2 before any
    # device work
    monkeypatch.setattr("sys.argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as e:
        bench.main()
    assert e.value.code == 2
    assert "exactly one GPU" in capsys.readouterr().err
