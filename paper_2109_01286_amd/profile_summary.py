"""Summarise rocprofv3 CSV output of a bench.py run into a short markdown
table (kernel statistics, and HBM traffic from FETCH_SIZE / WRITE_SIZE runs
calibrated on k_cast, a streaming kernel of known size: it reads 8 bytes and
writes 4 bytes per element).

    python -m paper_2109_01286_amd.profile_summary STATS_DIR FETCH_DIR WRITE_DIR OUT.md "COMMAND" [VALU_DIR [TA_DIR]]
    python -m paper_2109_01286_amd.profile_summary --stats STATS_DIR OUT.md "COMMAND" "TITLE"

VALU_DIR (optional) holds a ``--pmc VALUBusy`` run: the percentage of the
kernel's time the vector ALUs were busy, per hot-path kernel.  TA_DIR
(optional) holds a ``--pmc TA_BUSY_avr GRBM_GUI_ACTIVE`` run: the share of the
kernel's GPU cycles the texture addresser (the unit that takes every vector
memory instruction's addresses) was busy, averaged over its instances.

The second form writes the kernel statistics alone.
"""
import collections
import csv
import hashlib
import json
import os
import sys

KERNEL_SOURCES = [os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", f)
                  for f in ("kernels.hip", "gas.h")]


def source_digest():
    """sha256 of the hot-path kernel sources the counters belong to."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()


def _short(name):
    return name.replace("hfd::(anonymous namespace)::", "").replace("void ", "").split("(")[0]


def _agg(path, counter=None):
    rows = list(csv.DictReader(open(path)))
    a = collections.defaultdict(list)
    for r in rows:
        if counter is None or r["Counter_Name"] == counter:
            a[(_short(r["Kernel_Name"]), int(r["Grid_Size"]))].append(float(r["Counter_Value"]))
    return a


def _num_xcc(agent_csv):
    """XCD count of the GPU agent (1 if the agent file is absent)."""
    if not os.path.exists(agent_csv):
        return 1
    for r in csv.DictReader(open(agent_csv)):
        if r.get("Agent_Type") == "GPU" and r.get("Num_Xcc"):
            return max(1, int(r["Num_Xcc"]))
    return 1


def main(stats_dir, fetch_dir, write_dir, out, command, valu_dir=None, ta_dir=None):
    lines = ["# rocprofv3 summary: shock-vortex 2049 x 1025 (2.1 M owned vertices, 6.33 M active edges)", "",
             "Commands (on the MI355X box, from the repository root, `export TMPDIR=/tmp`):", "",
             *["    " + c.strip() for c in command.splitlines() if c.strip()], "",
             "## Kernel statistics (`--kernel-trace --stats`)", "",
             "| kernel | calls | average (ms) | min (ms) | max (ms) | share |", "|---|---|---|---|---|---|"]
    rows = list(csv.DictReader(open(os.path.join(stats_dir, "run_kernel_stats.csv"))))
    for r in rows[:14]:
        lines.append(f"| `{_short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e6:.4f} | "
                     f"{float(r['MinNs']) / 1e6:.4f} | {float(r['MaxNs']) / 1e6:.4f} | "
                     f"{float(r['Percentage']):.2f} % |")
    F = _agg(os.path.join(fetch_dir, "run_counter_collection.csv"))
    W = _agg(os.path.join(write_dir, "run_counter_collection.csv"))
    ck = max((k for k in F if k[0] == "k_cast"), key=lambda k: k[1])
    n = ck[1]
    ff = (8 * n / 1024) / (sum(F[ck]) / len(F[ck]))
    fw = (4 * n / 1024) / (sum(W[ck]) / len(W[ck]))
    lines += ["", "## HBM traffic per launch (`--pmc FETCH_SIZE`, then `--pmc WRITE_SIZE`)", "",
              f"Calibration on `k_cast` ({n} elements): FETCH_SIZE x {ff:.4f}, WRITE_SIZE x {fw:.4f}.", "",
              "| kernel | launches | fetch (GB) | write (GB) | total (GB) |", "|---|---|---|---|---|"]
    traffic = {}
    for k in sorted(F, key=lambda k: -sum(F[k])):
        if k[0].startswith(("k_vertex", "k_edge1<", "k_edge2<", "k_to_gather")):
            f = sum(F[k]) / len(F[k]) * 1024 * ff
            w = sum(W[k]) / len(W[k]) * 1024 * fw
            lines.append(f"| `{k[0]}` | {len(F[k])} | {f / 1e9:.3f} | {w / 1e9:.3f} | {(f + w) / 1e9:.3f} |")
            traffic[k[0]] = {"fetch_bytes": f, "write_bytes": w, "bytes": f + w}
    valu = {}
    if valu_dir:
        V = _agg(os.path.join(valu_dir, "run_counter_collection.csv"))
        lines += ["", "## Vector ALU busy (`--pmc VALUBusy`)", "",
                  "| kernel | launches | VALU busy (%) |", "|---|---|---|"]
        for k in sorted(V, key=lambda k: -sum(V[k])):
            if k[0].startswith(("k_vertex", "k_edge1<", "k_edge2<")):
                b = sum(V[k]) / len(V[k])
                lines.append(f"| `{k[0]}` | {len(V[k])} | {b:.1f} |")
                valu[k[0]] = b
    ta = {}
    if ta_dir:
        path = os.path.join(ta_dir, "run_counter_collection.csv")
        B, G = _agg(path, "TA_BUSY_avr"), _agg(path, "GRBM_GUI_ACTIVE")
        # GRBM_GUI_ACTIVE adds the busy cycles of every XCD's own GRBM
        nx = _num_xcc(os.path.join(ta_dir, "run_agent_info.csv"))
        lines += ["", "## Address unit busy (`--pmc TA_BUSY_avr GRBM_GUI_ACTIVE`)", "",
                  f"TA_BUSY_avr over GRBM_GUI_ACTIVE / {nx} (the XCD count).", "",
                  "| kernel | launches | TA busy (% of GPU cycles) |", "|---|---|---|"]
        for k in sorted(B, key=lambda k: -sum(B[k])):
            if k[0].startswith(("k_vertex", "k_edge1<", "k_edge2<")) and k in G:
                b = 100.0 * nx * sum(B[k]) / sum(G[k])
                lines.append(f"| `{k[0]}` | {len(B[k])} | {b:.1f} |")
                ta[k[0]] = b
    open(out, "w").write("\n".join(lines) + "\n")
    js = os.path.splitext(out)[0] + "_traffic.json"
    json.dump({"workload": "shockvortex2049", "kernel_sources_sha256": source_digest(),
               "fetch_factor": ff, "write_factor": fw, "per_launch": traffic,
               "valu_busy_percent": valu, "ta_busy_percent": ta},
              open(js, "w"), indent=1)


def stats_only(stats_dir, out, command, title):
    lines = [f"# rocprofv3 summary: {title}", "",
             "Commands (on the MI355X box, from the repository root, `export TMPDIR=/tmp`):", "",
             *["    " + c.strip() for c in command.splitlines() if c.strip()], "",
             "## Kernel statistics (`--kernel-trace --stats`)", "",
             "| kernel | calls | average (us) | min (us) | max (us) | share |", "|---|---|---|---|---|---|"]
    for r in csv.DictReader(open(os.path.join(stats_dir, "run_kernel_stats.csv"))):
        if float(r["Percentage"]) < 0.05:
            continue
        lines.append(f"| `{_short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                     f"{float(r['Percentage']):.2f} % |")
    open(out, "w").write("\n".join(lines) + "\n")


if __name__ == "__main__":
    if sys.argv[1] == "--stats":
        stats_only(*sys.argv[2:6])
    else:
        main(*sys.argv[1:8])
