"""Summarise rocprofv3 CSV output of profile_run into profiles/.

Usage:
    python -m paper_2011_06856_amd.profile_summary --stats DIR --fetch DIR --write DIR \
        --name stream_collide_f32_circular_1024 --command "..." --copy-mib 1024 \
        --launch-bytes 2147483648

Writes profiles/<name>.md (kernel timing table, counter readings, the copy
calibration factors and the derived HBM traffic per launch; without --fetch
and --write the timing table only, and with --step-kernels the kernel time
of one step summed over the kernels a step launches) and
profiles/<name>.json, which bench.py reads to fill its `traffic` field while
the kernel source is unchanged (sha256 of the kernel sources recorded here).
"""
import argparse
import csv
import glob
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
# The sources of the two step kernels and of what they read (tables, launch
# parameters): a summary taken on other versions of these is stale.  The
# network and batch code (mlp.hip, batch.cpp) do not enter the step kernels.
KERNEL_SOURCES = [os.path.join(HERE, "csrc", f)
                  for f in ("capi.cpp", "kernels.hip", "push.hip", "quadrature.cpp", "rlbm_internal.h")]


def kernel_source_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update(open(p, "rb").read())
    return h.hexdigest()


def _rows(d, suffix):
    files = glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True)
    rows = []
    for f in files:
        rows += list(csv.DictReader(open(f)))
    return rows


def counter_per_kernel(d, counter):
    out = {}
    for r in _rows(d, "counter_collection.csv"):
        if r["Counter_Name"] != counter:
            continue
        out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--stats", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--name", required=True)
    ap.add_argument("--command", required=True)
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--kernel", default="k_stream_collide")
    ap.add_argument("--launch-bytes", type=float, required=True, help="algorithmic bytes per launch")
    ap.add_argument("--out-dir", default=os.path.join(ROOT, "profiles"))
    ap.add_argument("--step-kernels", help="comma-separated kernel names whose launches make up one step")
    ap.add_argument("--steps", type=int, help="steps the traced run took (with --step-kernels)")
    ap.add_argument("--sv-per-step", type=float, help="site-velocity updates of one step (with --step-kernels)")
    ap.add_argument("--sq", nargs="*", default=[], help="rocprofv3 --pmc output dirs of SQ counter passes")
    ap.add_argument("--wave-units", type=float,
                    help="wave-velocities per launch (site-velocity updates / 64), for per-unit SQ counts")
    a = ap.parse_args()

    stats = _rows(a.stats, "kernel_stats.csv")
    fetch = counter_per_kernel(a.fetch, "FETCH_SIZE") if a.fetch else {}
    write = counter_per_kernel(a.write, "WRITE_SIZE") if a.write else {}
    copy_kib = a.copy_mib * 1024.0

    def pick(d, key):
        vals = [v for k, vs in d.items() if key in k.replace("(anonymous namespace)::", "") for v in vs]
        return vals

    kf, kw = pick(fetch, a.kernel), pick(write, a.kernel)
    cf, cw = max(pick(fetch, "copyBuffer") or [0]), max(pick(write, "copyBuffer") or [0])
    f_fac = copy_kib / cf if cf else None
    w_fac = copy_kib / cw if cw else None
    kf_avg = sum(kf) / len(kf) if kf else None
    kw_avg = sum(kw) / len(kw) if kw else None
    traffic = None
    if kf_avg and kw_avg and f_fac and w_fac:
        traffic = (kf_avg * f_fac + kw_avg * w_fac) * 1024.0
    kstat = [r for r in stats if a.kernel in r["Name"].replace("(anonymous namespace)::", "")]
    avg_ns = float(kstat[0]["AverageNs"]) if kstat else None

    lines = ["# %s" % a.name, "",
             "Command (run from the repository root on a machine with the GPU):", "", "```", a.command, "```", "",
             "## Kernel trace (rocprofv3 --kernel-trace --stats)", "",
             "| kernel | calls | avg us | min us | max us | % |", "|---|---|---|---|---|---|"]
    for r in sorted(stats, key=lambda r: -float(r["Percentage"])):
        nm = r["Name"].replace("(anonymous namespace)::", "").replace("void ", "").split("(")[0][:70]
        lines.append("| %s | %s | %.1f | %.1f | %.1f | %.1f |" % (nm, r["Calls"], float(r["AverageNs"]) / 1e3,
                                                                float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3,
                                                                float(r["Percentage"])))
    lines += [""]
    if a.fetch and a.write:
        lines += ["## HBM counters (rocprofv3 --pmc FETCH_SIZE, then --pmc WRITE_SIZE; KiB per dispatch)", "",
                  "| quantity | value |", "|---|---|",
                  "| calibration copy size | %d MiB read + %d MiB written |" % (a.copy_mib, a.copy_mib),
                  "| FETCH_SIZE of the copy | %s KiB -> factor %s |" % (cf, "%.4f" % f_fac if f_fac else "n/a"),
                  "| WRITE_SIZE of the copy | %s KiB -> factor %s |" % (cw, "%.4f" % w_fac if w_fac else "n/a"),
                  "| %s FETCH_SIZE (avg of %d) | %s KiB |" % (a.kernel, len(kf), "%.1f" % kf_avg if kf_avg else "n/a"),
                  "| %s WRITE_SIZE (avg of %d) | %s KiB |" % (a.kernel, len(kw), "%.1f" % kw_avg if kw_avg else "n/a"),
                  "| traffic per launch (scaled) | %s bytes |" % ("%.4g" % traffic if traffic else "n/a"),
                  "| algorithmic bytes per launch | %.4g |" % a.launch_bytes,
                  "| traffic / algorithmic | %s |" % ("%.3f" % (traffic / a.launch_bytes) if traffic else "n/a"),
                  "| avg launch duration | %s us |" % ("%.1f" % (avg_ns / 1e3) if avg_ns else "n/a"),
                  "| algorithmic GB/s at that duration | %s |" % ("%.0f" % (a.launch_bytes / avg_ns) if avg_ns else "n/a"),
                  ""]
    sq = {}
    for d in a.sq:
        for r in _rows(d, "counter_collection.csv"):
            if a.kernel not in r["Kernel_Name"].replace("(anonymous namespace)::", ""):
                continue
            sq.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    if sq:
        avg = {k: sum(v) / len(v) for k, v in sq.items()}
        lines += ["## Instruction mix and wave states (rocprofv3 --pmc, SQ counters, averages per launch)", "",
                  "| counter | per launch | per wave-velocity |", "|---|---|---|"]
        for k in sorted(avg):
            per = ("%.2f" % (avg[k] / a.wave_units)) if (a.wave_units and k.startswith("SQ_INSTS")) else ""
            lines.append("| %s | %.4g | %s |" % (k, avg[k], per))
        wc = avg.get("SQ_WAVE_CYCLES")
        if wc:
            lines += ["", "| wave state | fraction of wave cycles |", "|---|---|"]
            for k, label in (("SQ_WAIT_INST_ANY", "waiting on an issued instruction's result (memory counters)"),
                             ("SQ_WAIT_ANY", "waiting on anything"),
                             ("SQ_ACTIVE_INST_ANY", "issuing any instruction"),
                             ("SQ_ACTIVE_INST_VALU", "issuing VALU"),
                             ("SQ_ACTIVE_INST_SCA", "issuing scalar"),
                             ("SQ_ACTIVE_INST_LDS", "issuing LDS")):
                if k in avg:
                    lines.append("| %s (%s) | %.3f |" % (k, label, avg[k] / wc))
        lines += [""]
    if a.step_kernels and a.steps and a.sv_per_step:
        names = a.step_kernels.split(",")
        step_rows = [r for r in stats if any(k in r["Name"] for k in names)]
        per_step_ns = sum(float(r["TotalDurationNs"]) for r in step_rows) / a.steps
        lines += ["## One step", "",
                  "| quantity | value |", "|---|---|",
                  "| kernels of a step | %s |" % ", ".join("%s (%s calls)" % (
                      r["Name"].replace("(anonymous namespace)::", "").replace("void ", "").split("(")[0], r["Calls"])
                      for r in step_rows),
                  "| kernel time per step (sum over those kernels / %d steps) | %.1f us |" % (a.steps, per_step_ns / 1e3),
                  "| site-velocity updates per step | %.6g |" % a.sv_per_step,
                  "| GSVUPS at that time | %.1f |" % (a.sv_per_step / per_step_ns),
                  "| algorithmic GB/s at 8 B a site-velocity | %.0f |" % (8.0 * a.sv_per_step / per_step_ns), ""]
    lines += ["Kernel sources sha256: `%s`" % kernel_source_hash(), ""]
    os.makedirs(a.out_dir, exist_ok=True)
    md = os.path.join(a.out_dir, a.name + ".md")
    open(md, "w").write("\n".join(lines))
    js = dict(name=a.name, command=a.command, kernel=a.kernel, avg_launch_ns=avg_ns, traffic_bytes=traffic,
              fetch_kib=kf_avg, write_kib=kw_avg, fetch_factor=f_fac, write_factor=w_fac,
              launch_bytes=a.launch_bytes, kernel_sha256=kernel_source_hash())
    json.dump(js, open(os.path.join(a.out_dir, a.name + ".json"), "w"), indent=1)
    print(md)


if __name__ == "__main__":
    main()
