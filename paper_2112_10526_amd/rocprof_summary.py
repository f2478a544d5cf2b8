"""Summaries of rocprofv3 output for the profiles folder: kernel-time tables,
HBM traffic per launch from FETCH_SIZE / WRITE_SIZE counter runs (scaled by a
plain copy of known size), wave-state and matrix-core counter tables.

Usage (each prints or writes one markdown summary):
  python -m paper_2112_10526_amd.rocprof_summary stats KERNEL_STATS_CSV CMD TITLE
  python -m paper_2112_10526_amd.rocprof_summary mfma COUNTER_DIR CMD TITLE
  python -m paper_2112_10526_amd.rocprof_summary waves COUNTER_DIR CMD [TITLE]
  python -m paper_2112_10526_amd.rocprof_summary traffic FETCH_DIR WRITE_DIR CLASS PRECISION \
      COPY_MIB FETCH_CMD WRITE_CMD
"""
from __future__ import annotations

import collections
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
PROFILES = os.path.join(os.path.dirname(HERE), "profiles")

# kernel class -> (source file of its kernel, symbol prefix in profiles)
KERNELS = {  # (BF16 form, the benchmark's main run)
    "qgt_w": ("qgt.hip", "k_w7"), "outer": ("qgt.hip", "k_outer8"),
    "reduce": ("qgt.hip", "k_update5"),
    "sample": ("sampler.hip", "k_sample<float"), "eloc": ("eloc.hip", "k_eloc<float"),
    "theta": ("theta.hip", "k_theta_bf16"),
}


def source_digest(cls: str) -> str:
    """Digest of the sources a kernel class is built from (its file + shared headers)."""
    import hashlib
    h = hashlib.sha256()
    for f in ("common.h", "kernels.h", KERNELS.get(cls, ("qgt.hip",))[0]):
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_file(cls: str, precision: str) -> str:
    sym = KERNELS.get(cls, (None, cls))[1].split("<")[0]
    return os.path.join(PROFILES, f"traffic_{sym}_tfim2d_l10_{precision}.md")


def read_traffic(cls: str, precision: str):
    """HBM bytes per launch from the committed counter summary, or None when it is
    missing or was taken on other kernel sources."""
    path = traffic_file(cls, precision)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].split(": ", 1)
                kv[k.strip()] = v.strip().strip("`")
    if kv.get("source_digest") != source_digest(cls):
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _counter_rows(d):
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            rows += list(csv.DictReader(fh))
    if not rows:
        raise SystemExit(f"no counter_collection.csv under {d}")
    return rows


def _per_dispatch(rows, counter, match):
    """Mean over dispatches of kernels whose name contains `match` of the counter (summed
    over its instances within one dispatch).  Dispatches below a tenth of the largest one
    are left out: they are the CG launches queued after a solve had stopped, which
    return at once."""
    per = {}
    for r in rows:
        if r.get("Counter_Name") != counter or match not in r.get("Kernel_Name", ""):
            continue
        key = r.get("Dispatch_Id") or r.get("Correlation_Id")
        per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
    if not per:
        names = sorted({r.get("Kernel_Name", "")[:80] for r in rows})
        raise SystemExit(f"no {counter} rows for a kernel matching {match!r}; kernels: {names}")
    vals = np.array(list(per.values()))
    vals = vals[vals >= 0.1 * vals.max()]
    return float(vals.mean()), len(vals)


def summarize_traffic(fetch_dir, write_dir, cls, precision, copy_mib, cmds):
    """Write the traffic summary of one kernel class from two counter runs (FETCH_SIZE,
    WRITE_SIZE; KiB per dispatch), each scaled by the same counter on a plain copy of
    copy_mib MiB (torch's elementwise multiply by 1: one read, one write)."""
    sym = KERNELS[cls][1]
    fr, wr = _counter_rows(fetch_dir), _counter_rows(write_dir)
    copy_bytes = copy_mib * 2.0 ** 20
    cf, _ = _per_dispatch(fr, "FETCH_SIZE", "MulFunctor")
    cw, _ = _per_dispatch(wr, "WRITE_SIZE", "MulFunctor")
    kf, nf = _per_dispatch(fr, "FETCH_SIZE", sym)
    kw, nw = _per_dispatch(wr, "WRITE_SIZE", sym)
    f_scale, w_scale = copy_bytes / cf, copy_bytes / cw
    fetch_b, write_b = kf * f_scale, kw * w_scale
    lines = [
        f"# HBM traffic of `{sym}` (10x10 TFIM workload, {precision})", "",
        "Two rocprofv3 counter runs of the same command, one counter each:", "",
        f"    {cmds[0]}", f"    {cmds[1]}", "",
        f"Counters are KiB per dispatch; each is scaled by what it reads for a plain copy of "
        f"{copy_mib} MiB (torch elementwise multiply by 1, one read and one write) run in the "
        f"same process.", "",
        f"- kernel_class: {cls}",
        f"- source_digest: `{source_digest(cls)}`",
        f"- copy_fetch_kib: {cf:.1f}", f"- copy_write_kib: {cw:.1f}",
        f"- fetch_scale: {f_scale:.4f}", f"- write_scale: {w_scale:.4f}",
        f"- dispatches counted: {nf} (fetch run), {nw} (write run)",
        f"- fetch_kib_per_launch: {kf:.1f}", f"- write_kib_per_launch: {kw:.1f}",
        f"- fetch_bytes_per_launch: {fetch_b:.0f}", f"- write_bytes_per_launch: {write_b:.0f}",
        f"- hbm_bytes_per_launch: {fetch_b + write_b:.0f}",
    ]
    path = traffic_file(cls, precision)
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(path)


def summarize_waves(counter_dir, cmd,
                    title="Wave-state counters of the hot-path kernels (10x10 TFIM workload, "
                          "BF16 form)"):
    """Markdown table of the wave-state counters (SQ_*) of the hot-path kernels."""
    rows = _counter_rows(counter_dir)
    agg = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in rows:
        name = r["Kernel_Name"].split("(")[0].replace("void ", "")
        agg[name][r["Counter_Name"]].append(float(r["Counter_Value"]))
    out = [f"# {title}", "",
           "Command:", "", "    " + cmd, "",
           "Median over the dispatches of one kernel (dispatches that return at once after a "
           "CG solve has stopped are left out); WAVE_CYCLES, WAIT_* and ACTIVE_* are summed "
           "over waves.", "",
           "| kernel | waves | wave cycles / wave | wait (memory) % | wait (issue) % | active % |",
           "|---|---:|---:|---:|---:|---:|"]
    for name in ["nqs::k_w7", "nqs::k_outer8", "nqs::k_update5<",
                 "nqs::k_sample<float, 4, 0, 2>", "nqs::k_sample<float, 16, 1, 1>",
                 "nqs::k_eloc<float, 0>", "nqs::k_eloc<float, 1>", "nqs::k_theta_bf16",
                 "nqs::k_w5", "nqs::k_outer9<", "nqs::k_update4<",
                 "nqs::k_sample<double, 4, 0, 2>", "nqs::k_sample<double, 16, 1, 1>",
                 "nqs::k_eloc<double, 0>", "nqs::k_eloc<double, 1>", "nqs::k_theta<double>"]:
        # (a name ending in "<" stands for every instantiation of that template)
        hits = [k for k in agg if k.startswith(name)] if name.endswith("<") else (
            [name] if name in agg else [])
        for name in sorted(hits):
            _wave_row(out, name, agg[name])
    print("\n".join(out))


def _wave_row(out, name, d):
    """One row of the wave-state table: medians over the dispatches that did work."""
    wc = np.array(d["SQ_WAVE_CYCLES"])
    keep = wc >= 0.1 * wc.max()
    med = {k: float(np.median(np.array(v)[keep])) for k, v in d.items() if len(v) == len(wc)}
    w = med["SQ_WAVE_CYCLES"]
    out.append(f"| `{name}` | {med['SQ_WAVES']:.0f} | {w / med['SQ_WAVES']:.0f} | "
               f"{100 * med['SQ_WAIT_ANY'] / w:.0f} | {100 * med['SQ_WAIT_INST_ANY'] / w:.0f} | "
               f"{100 * med['SQ_ACTIVE_INST_ANY'] / w:.0f} |")


MFMA_COUNTERS = ("SQ_INSTS_VALU_MFMA_MOPS_BF16", "SQ_INSTS_VALU_MFMA_MOPS_F32",
                 "SQ_INSTS_VALU_MFMA_MOPS_F64", "SQ_VALU_MFMA_BUSY_CYCLES", "SQ_BUSY_CU_CYCLES",
                 "GRBM_GUI_ACTIVE")


def summarize_mfma(counter_dir, cmd, title, n_cu=256, n_xcd=8):
    """Markdown table of matrix-core counters per kernel: MFMA operations (the MOPS
    counters count flops / 512), matrix-core busy cycles and their share of the
    kernel's GPU-active cycles over all SIMDs,
    util = SQ_VALU_MFMA_BUSY_CYCLES (summed over SIMDs) / (GRBM_GUI_ACTIVE / XCDs x CUs x 4):
    rocprofv3 reports GRBM_GUI_ACTIVE summed over the eight XCDs, each of which counts the
    kernel's active cycles (eight times 188 ms at the 2.4 GHz clock for a 188 ms kernel)."""
    rows = _counter_rows(counter_dir)
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    names = {}
    for r in rows:
        key = r.get("Dispatch_Id") or r.get("Correlation_Id")
        name = r["Kernel_Name"].split("(")[0].replace("void ", "")
        names[key] = name
        per[key][r["Counter_Name"]] += float(r["Counter_Value"])
    agg = collections.defaultdict(list)
    for key, c in per.items():
        mops = sum(c.get(k, 0.0) for k in MFMA_COUNTERS[:3])
        if mops > 0:
            agg[names[key]].append(c)
    out = [f"# {title}", "", "Command:", "", "    " + cmd, "",
           "Per kernel, median over its dispatches that issued matrix-core work (CG launches "
           "queued after a solve stopped are left out: under a tenth of the largest). "
           "`flop` = MOPS x 512 (the MOPS counters count operations / 512); "
           f"`MFMA busy %` = SQ_VALU_MFMA_BUSY_CYCLES (summed over SIMDs) / (GRBM_GUI_ACTIVE "
           f"/ {n_xcd} x {n_cu} CUs x 4 SIMDs): GRBM_GUI_ACTIVE comes summed over the "
           f"{n_xcd} XCDs, each counting the kernel's active cycles.", "",
           "| kernel | dispatches | flop (BF16) | flop (FP32) | flop (FP64) | MFMA busy cycles | "
           "GUI active cycles | MFMA busy % |",
           "|---|---:|---:|---:|---:|---:|---:|---:|"]
    for name in sorted(agg, key=lambda k: -np.median([c["SQ_VALU_MFMA_BUSY_CYCLES"]
                                                       for c in agg[k]])):
        cs = agg[name]
        tot = np.array([sum(c.get(k, 0.0) for k in MFMA_COUNTERS[:3]) for c in cs])
        keep = tot >= 0.1 * tot.max()
        cs = [c for c, k in zip(cs, keep) if k]
        med = {k: float(np.median([c.get(k, 0.0) for c in cs])) for k in MFMA_COUNTERS}
        util = med["SQ_VALU_MFMA_BUSY_CYCLES"] / max(med["GRBM_GUI_ACTIVE"] / n_xcd * n_cu * 4, 1.0)
        out.append(f"| `{name}` | {len(cs)} | {512 * med['SQ_INSTS_VALU_MFMA_MOPS_BF16']:.4g} | "
                   f"{512 * med['SQ_INSTS_VALU_MFMA_MOPS_F32']:.4g} | "
                   f"{512 * med['SQ_INSTS_VALU_MFMA_MOPS_F64']:.4g} | "
                   f"{med['SQ_VALU_MFMA_BUSY_CYCLES']:.4g} | {med['GRBM_GUI_ACTIVE']:.4g} | "
                   f"{100 * util:.1f} |")
    print("\n".join(out))


def _full_launch_medians(trace_csv):
    """Per kernel: median duration (us) and count of the launches that did the work.
    CG kernels queued after the solve has stopped return at once; launches shorter
    than 30 % of the kernel's 90th-percentile duration are left out."""
    import csv
    durs = collections.defaultdict(list)
    with open(trace_csv) as fh:
        for r in csv.DictReader(fh):
            name = r["Kernel_Name"].split("(")[0].replace("void ", "")
            durs[name].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    out = {}
    for name, v in durs.items():
        a = np.array(v)
        full = a[a >= 0.3 * np.percentile(a, 90)]
        out[name] = (float(np.median(full)), len(full))
    return out


def summarize_stats(stats_csv, cmd, title):
    """Markdown table of a rocprofv3 kernel_stats.csv (with the median of the full
    launches from the kernel_trace.csv beside it, when present)."""
    import csv
    with open(stats_csv) as fh:
        rows = list(csv.DictReader(fh))
    trace = stats_csv.replace("kernel_stats.csv", "kernel_trace.csv")
    med = _full_launch_medians(trace) if os.path.exists(trace) else {}
    out = [f"# {title}", "", "Command:", "", f"    {cmd}", "",
           "`full med us`: median duration of the launches that did the work (CG kernels "
           "queued after a solve has stopped return at once; launches under 30 % of the "
           "kernel's 90th-percentile duration are left out), over `full` launches.", "",
           "| kernel | calls | avg us | min us | max us | total ms | % | full | full med us |",
           "|---|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for r in rows:
        name = r["Name"].split("(")[0].replace("void ", "")
        m, c = med.get(name, (float("nan"), 0))
        out.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                   f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
                   f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.2f} | "
                   f"{c} | {m:.2f} |")
    if os.path.exists(trace):
        span, busy, n = _trace_span(trace)
        out += ["", f"Trace: {n} launches; span from the first start to the last end "
                    f"{span / 1e6:.1f} ms; kernel time summed over all streams {busy / 1e6:.1f} ms "
                    f"({100.0 * busy / span:.0f} % of the span)."]
    print("\n".join(out))


def _trace_span(trace_csv):
    import csv
    t0, t1, busy, n = None, None, 0, 0
    with open(trace_csv) as fh:
        for r in csv.DictReader(fh):
            a, b = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
            t0 = a if t0 is None else min(t0, a)
            t1 = b if t1 is None else max(t1, b)
            busy += b - a
            n += 1
    return (t1 - t0 if n else 0), busy, n


def main(argv=None):
    argv = list(sys.argv[1:] if argv is None else argv)
    if not argv:
        print(__doc__)
        return 2
    cmd, rest = argv[0], argv[1:]
    if cmd == "stats":
        summarize_stats(*rest)
    elif cmd == "mfma":
        summarize_mfma(*rest)
    elif cmd == "waves":
        summarize_waves(*rest)
    elif cmd == "traffic":
        fd, wd, cls, prec, mib, c1, c2 = rest
        summarize_traffic(fd, wd, cls, prec, int(mib), (c1, c2))
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main())
