"""The rocprofv3 summariser on synthetic CSV files: the FETCH_SIZE and
WRITE_SIZE scale factors come from the plain streaming kernel (k_cast reads 8
and writes 4 bytes per element), every hot-path kernel's counters are scaled
by them, and the VALU and address-unit tables take each counter's own rows
(the GPU cycles counted once per XCD)."""
import csv
import json
import os

from paper_2109_01286_amd import profile_summary as P

VERTEX = "void hfd::(anonymous namespace)::k_vertex<float, false, 1>(long, long)"
EDGE = "void hfd::(anonymous namespace)::k_edge1<float>(long)"
CAST = "hfd::(anonymous namespace)::k_cast(long, double const*, float*)"


def _counters(path, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, ["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, grid, counter, value in rows:
            w.writerow({"Kernel_Name": name, "Grid_Size": grid, "Counter_Name": counter,
                        "Counter_Value": value})


def test_traffic_is_calibrated_on_the_streaming_kernel(tmp_path):
    n = 1 << 20
    stats = tmp_path / "stats"
    stats.mkdir()
    with open(stats / "run_kernel_stats.csv", "w", newline="") as f:
        w = csv.DictWriter(f, ["Name", "Calls", "AverageNs", "MinNs", "MaxNs", "Percentage"])
        w.writeheader()
        w.writerow({"Name": VERTEX, "Calls": 3, "AverageNs": 660000, "MinNs": 650000,
                    "MaxNs": 670000, "Percentage": 70.0})
    # the counters read half of the bytes read and all of the bytes written
    _counters(str(tmp_path / "f"), [(CAST, n, "FETCH_SIZE", 8 * n / 1024 / 2),
                                    (VERTEX, 4096, "FETCH_SIZE", 1000.0),
                                    (VERTEX, 4096, "FETCH_SIZE", 1200.0)])
    _counters(str(tmp_path / "w"), [(CAST, n, "WRITE_SIZE", 4 * n / 1024),
                                    (VERTEX, 4096, "WRITE_SIZE", 50.0),
                                    (VERTEX, 4096, "WRITE_SIZE", 50.0)])
    _counters(str(tmp_path / "v"), [(VERTEX, 4096, "VALUBusy", 60.0), (EDGE, 512, "VALUBusy", 40.0)])
    _counters(str(tmp_path / "t"), [(VERTEX, 4096, "TA_BUSY_avr", 300.0),
                                    (VERTEX, 4096, "GRBM_GUI_ACTIVE", 1000.0),
                                    (EDGE, 512, "TA_BUSY_avr", 50.0),
                                    (EDGE, 512, "GRBM_GUI_ACTIVE", 200.0)])
    # GRBM_GUI_ACTIVE adds the cycles of every XCD: here two
    with open(tmp_path / "t" / "run_agent_info.csv", "w", newline="") as f:
        w = csv.DictWriter(f, ["Agent_Type", "Num_Xcc"])
        w.writeheader()
        w.writerow({"Agent_Type": "CPU", "Num_Xcc": 0})
        w.writerow({"Agent_Type": "GPU", "Num_Xcc": 2})
    out = str(tmp_path / "summary.md")
    P.main(str(stats), str(tmp_path / "f"), str(tmp_path / "w"), out, "cmd", str(tmp_path / "v"),
           str(tmp_path / "t"))
    js = json.load(open(str(tmp_path / "summary_traffic.json")))
    assert abs(js["fetch_factor"] - 2.0) < 1e-12 and abs(js["write_factor"] - 1.0) < 1e-12
    v = js["per_launch"]["k_vertex<float, false, 1>"]
    assert abs(v["fetch_bytes"] - 1100.0 * 1024 * 2) < 1e-6
    assert abs(v["write_bytes"] - 50.0 * 1024) < 1e-6
    assert js["valu_busy_percent"] == {"k_vertex<float, false, 1>": 60.0, "k_edge1<float>": 40.0}
    assert js["ta_busy_percent"] == {"k_vertex<float, false, 1>": 60.0, "k_edge1<float>": 50.0}
    assert js["kernel_sources_sha256"] == P.source_digest()
    text = open(out).read()
    assert "| `k_vertex<float, false, 1>` | 3 | 0.6600 |" in text
