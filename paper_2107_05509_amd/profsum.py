"""Summaries of rocprofv3 output for this library's kernels (host-side tool,
no GPU needed).

  python -m paper_2107_05509_amd.profsum stats  <run_kernel_stats.csv> --cmd "..." --title "..."
  python -m paper_2107_05509_amd.profsum pmc    <run_counter_collection.csv>... --cmd "..." --title "..."
  python -m paper_2107_05509_amd.profsum traffic <fetch.csv> <write.csv> --cmd "..." --title "..."
                                                [--json profiles/traffic.json]

`stats` keeps the kernel-trace statistics rows of the hr:: kernels.  `pmc`
averages every counter per dispatch and kernel and adds derived ratios when
their counters are present (VALU lane utilisation = SQ_THREAD_CYCLES_VALU /
(64 SQ_ACTIVE_INST_VALU); waiting share = SQ_WAIT_ANY / SQ_WAVE_CYCLES;
instructions per wave).  `traffic` turns FETCH_SIZE and WRITE_SIZE (KiB per
dispatch) into HBM bytes: each counter is scaled by what it reads for the
calibration copy in the same run (the largest `__amd_rocclr_copyBuffer`
dispatches, a device copy of CAL_BYTES in and CAL_BYTES out, far beyond the
caches), and writes the per-launch bytes with the kernel sources' hash to the
JSON file the benchmark reads.  Every summary states the command it came from.
"""
import argparse
import collections
import csv
import json
import sys

from .build import source_hash

CAL_BYTES = 512 << 20   # the benchmark's calibration copy: 2^27 float32 in and out


def _short(name):
    n = name.split("(")[0]
    return n.replace("void ", "").replace("hr::", "")


def _header(title, cmd, out):
    out.append(f"# {title}")
    out.append(f"# source hash of the HIP kernels: {source_hash()}")
    for c in cmd:
        out.append(f"# command: {c}")


def stats(path, title, cmd):
    rows = list(csv.DictReader(open(path)))
    out = []
    _header(title, cmd, out)
    out.append("Name,Calls,AverageNs,MinNs,MaxNs,StdDev,Percentage")
    for r in rows:
        if "hr::" not in r["Name"]:
            continue
        out.append(",".join([_short(r["Name"]), r["Calls"], f"{float(r['AverageNs']):.0f}", r["MinNs"], r["MaxNs"],
                             f"{float(r['StdDev']):.0f}", f"{float(r['Percentage']):.2f}"]))
    return "\n".join(out) + "\n"


def _per_dispatch(paths):
    """{kernel: {counter: mean over dispatches}}, {kernel: dispatches}"""
    acc = collections.defaultdict(lambda: collections.defaultdict(float))
    seen = collections.defaultdict(set)
    for p in paths:
        for r in csv.DictReader(open(p)):
            k = _short(r["Kernel_Name"])
            key = (p, r["Dispatch_Id"])
            acc[k][r["Counter_Name"]] += float(r["Counter_Value"])
            seen[k].add(key)
    n = {k: len(v) for k, v in seen.items()}
    mean = {}
    for k, c in acc.items():
        # each dispatch appears once per file that holds its counters
        per_file = collections.Counter(p for p, _ in seen[k])
        mean[k] = {name: v / max(1, min(per_file.values())) for name, v in c.items()}
    return mean, n


def pmc(paths, title, cmd):
    mean, n = _per_dispatch(paths)
    out = []
    _header(title, cmd, out)
    out.append("# per dispatch, averaged over the run's dispatches of each kernel")
    for k in sorted(mean):
        if not (k.startswith("k_") and "<true>" not in k):
            continue
        c = mean[k]
        parts = [f"{name}={v:.0f}" for name, v in sorted(c.items())]
        if c.get("SQ_ACTIVE_INST_VALU"):
            if "SQ_THREAD_CYCLES_VALU" in c:
                parts.append(f"valu_lane_util={c['SQ_THREAD_CYCLES_VALU'] / (64.0 * c['SQ_ACTIVE_INST_VALU']):.3f}")
        if c.get("SQ_WAVE_CYCLES") and "SQ_WAIT_ANY" in c:
            parts.append(f"wait_share={c['SQ_WAIT_ANY'] / c['SQ_WAVE_CYCLES']:.3f}")
        if c.get("SQ_WAVES"):
            for name in ("SQ_INSTS_VALU", "SQ_INSTS_SALU"):
                if name in c:
                    parts.append(f"{name}_per_wave={c[name] / c['SQ_WAVES']:.0f}")
        out.append(f"{k}: " + ", ".join(parts))
    return "\n".join(out) + "\n"


def _counter(path, name):
    """{kernel: mean counter value per dispatch}, calibration value"""
    per = collections.defaultdict(list)
    cal = []
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != name:
            continue
        v = float(r["Counter_Value"])
        if r["Kernel_Name"].startswith("__amd_rocclr_copyBuffer"):
            cal.append(v)
        per[_short(r["Kernel_Name"])].append(v)
    if not cal:
        raise SystemExit(f"{path}: no calibration copy found")
    top = sorted(cal)[-3:]   # the calibration copies are the largest copies of the run
    return {k: sum(v) / len(v) for k, v in per.items()}, sum(top) / len(top)


def traffic(fetch_csv, write_csv, title, cmd):
    f, fcal = _counter(fetch_csv, "FETCH_SIZE")
    w, wcal = _counter(write_csv, "WRITE_SIZE")
    fs, ws = CAL_BYTES / (fcal * 1024.0), CAL_BYTES / (wcal * 1024.0)
    out = []
    _header(title, cmd, out)
    out.append(f"# scale: the calibration copy ({CAL_BYTES} B in and out) reads FETCH_SIZE {fcal:.1f} KiB -> x{fs:.3f}, "
               f"WRITE_SIZE {wcal:.1f} KiB -> x{ws:.3f}")
    out.append("kernel,FETCH_SIZE_KiB,WRITE_SIZE_KiB,scaled_read_MB,scaled_write_MB,scaled_total_MB")
    js = {"source_hash": source_hash(), "units": "bytes per launch (counter values scaled by the copy kernel)",
          "scale": {"fetch": fs, "write": ws}, "kernels": {}, "detail": {}}
    for k in sorted(set(f) | set(w)):
        # the counting instantiations (<true ...>) are not launched in the
        # timed region; the others keep their plain name
        if not (k.startswith("k_") and "<true" not in k):
            continue
        kk = k.replace("<false>", "").replace("<false, false>", "")
        rb, wb = f.get(k, 0.0) * 1024.0 * fs, w.get(k, 0.0) * 1024.0 * ws
        out.append(f"{kk},{f.get(k, 0.0):.1f},{w.get(k, 0.0):.1f},{rb / 1e6:.2f},{wb / 1e6:.2f},{(rb + wb) / 1e6:.2f}")
        js["kernels"][kk] = int(rb + wb)
        js["detail"][kk] = {"read_bytes": rb, "write_bytes": wb}
    return "\n".join(out) + "\n", js


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=("stats", "pmc", "traffic"))
    ap.add_argument("csv", nargs="+")
    ap.add_argument("--cmd", action="append", default=[])
    ap.add_argument("--title", default="")
    ap.add_argument("--json", default=None)
    a = ap.parse_args(argv)
    if a.mode == "stats":
        sys.stdout.write(stats(a.csv[0], a.title, a.cmd))
    elif a.mode == "pmc":
        sys.stdout.write(pmc(a.csv, a.title, a.cmd))
    else:
        text, js = traffic(a.csv[0], a.csv[1], a.title, a.cmd)
        js["workload"] = a.title
        sys.stdout.write(text)
        if a.json:
            json.dump(js, open(a.json, "w"), indent=1)


if __name__ == "__main__":
    main()
