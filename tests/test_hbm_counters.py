"""Host logic of the HBM counter reduction (no GPU): calibration by the copy
launch, selection of NVE-phase launches, the source digest gate."""
import csv
import json
import os

from paper_0809_2811_amd import hbm_counters


def _write(directory, counter, rows):
    os.makedirs(os.path.join(directory, "host", "1"), exist_ok=True)
    path = os.path.join(directory, "host", "1", "run_counter_collection.csv")
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for k, (name, val) in enumerate(rows):
            w.writerow({"Dispatch_Id": k + 1, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": val})


def test_reduce_scales_and_selects(tmp_path):
    mom, frc = "void k_moments<8, false>(Dev, Phys, int, int)", "void k_forces<8, 2, false>(Dev, Phys, int)"
    kick = "void k_forces<8, 4, false>(Dev, Phys, int)"
    seq_f = [("neg_kernel", 524288.0), (mom, 999.0), (kick, 999.0),   # melt: moments followed by a kick
             (mom, 100.0), (frc, 200.0), (mom, 300.0), (frc, 400.0)]
    seq_w = [("neg_kernel", 1048576.0), (mom, 9.0), (kick, 9.0), (mom, 10.0), (frc, 20.0), (mom, 30.0), (frc, 40.0)]
    _write(str(tmp_path / "f"), "FETCH_SIZE", seq_f)
    _write(str(tmp_path / "w"), "WRITE_SIZE", seq_w)
    out = str(tmp_path / "rec.json")
    rec = hbm_counters.reduce(str(tmp_path / "f"), str(tmp_path / "w"), out)
    assert rec["fetch_scale"] == 2.0 and rec["write_scale"] == 1.0
    k = rec["kernels"]
    assert k["liquid262144/k_moments<8, false>"] == {"fetch_bytes": 200.0 * 1024, "write_bytes": 20.0 * 1024,
                                                     "launches": 2}
    assert k["liquid262144/k_forces<8, 2, false>"]["fetch_bytes"] == 300.0 * 1024
    assert set(k) == {"liquid262144/k_moments<8, false>", "liquid262144/k_forces<8, 2, false>"}
    assert json.load(open(out))["kernel_sources_sha256"] == hbm_counters.kernel_sources_digest()


def test_traffic_only_for_current_sources(tmp_path, monkeypatch):
    rec = {"kernel_sources_sha256": "0" * 64, "fetch_scale": 2.0, "write_scale": 1.0,
           "kernels": {"liquid4096/k": {"fetch_bytes": 10.0, "write_bytes": 5.0, "launches": 1}}}
    path = tmp_path / "rec.json"
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(hbm_counters, "RECORD", str(path))
    assert hbm_counters.measured_traffic("k", "liquid4096") is None
    rec["kernel_sources_sha256"] = hbm_counters.kernel_sources_digest()
    path.write_text(json.dumps(rec))
    assert hbm_counters.measured_traffic("k", "liquid4096") == 25.0
    assert hbm_counters.measured_traffic("other", "liquid4096") is None


def _write_trace(directory, durations_ns):
    path = os.path.join(directory, "host", "1", "run_kernel_trace.csv")
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for k, d in enumerate(durations_ns):
            w.writerow({"Dispatch_Id": k + 1, "Start_Timestamp": 1000 * k, "End_Timestamp": 1000 * k + d})


def test_moments_split_into_rebuild_and_plain_launches(tmp_path):
    """With the run's kernel trace beside the counters, k_moments launches
    split at the midpoint of their (bimodal) durations; the plain average
    over all of them stays as before."""
    mom, frc = "void k_moments<8, false>(Dev, Phys, int, int)", "void k_forces<8, 2, false>(Dev, Phys, int)"
    seq = [("neg_kernel", 1048576.0), (mom, 70.0), (frc, 5.0), (mom, 20.0), (frc, 5.0), (mom, 74.0), (frc, 5.0)]
    dur = [500, 72000, 31000, 20000, 31000, 76000, 31000]
    for sub, counter in (("f", "FETCH_SIZE"), ("w", "WRITE_SIZE")):
        _write(str(tmp_path / sub), counter, seq)
        _write_trace(str(tmp_path / sub), dur)
    rec = hbm_counters.reduce(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "rec.json"))
    k = rec["kernels"]
    base = "liquid262144/k_moments<8, false>"
    assert k[base]["launches"] == 3 and abs(k[base]["fetch_bytes"] - 164.0 / 3 * 1024) < 1e-6
    assert k[base + "/rebuild"] == {"fetch_bytes": 72.0 * 1024, "write_bytes": 72.0 * 1024, "launches": 2}
    assert k[base + "/plain"] == {"fetch_bytes": 20.0 * 1024, "write_bytes": 20.0 * 1024, "launches": 1}
    assert "liquid262144/k_forces<8, 2, false>/rebuild" not in k
