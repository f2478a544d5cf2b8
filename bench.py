#!/usr/bin/env python3
"""Benchmark of the RBM-VMC hot path on the 10x10 transverse-field Ising model.

Workload (synthetic, seeded): 2D TFIM on a periodic 10 x 10 lattice, J = 1,
h = 3.044; real RBM with alpha = 2 (200 hidden units, 20,300 parameters),
initial parameters N(0, 0.01^2) from seed 1; Metropolis-local sampling with
4096 chains x 4 samples per SR step (16,384 samples), 100 proposals between
recorded samples; SR with the on-the-fly QGT product, CG tolerance 1e-6,
diagonal shift 0.01, learning rate 0.01.  The chains are thermalised for
100 x 100 proposals before timing (not timed).

One timed "step" = one full SR step: sampling, local energies, statistics,
force, CG solve and parameter update.  `value` is the BF16 form's end-to-end
local energies per second (samples x SR steps / s); the FP64 path is timed the
same way and reported beside it.  For the roofline figure the same number of
steps is then run again with every launch of the dominant kernel class
bracketed by HIP events on the stream it runs on (event timing needs the CG
kernels launched one by one, so this pass does not replay CG graphs and is
not the one `value` comes from; its step time is reported too).
"""
from __future__ import annotations

import argparse
import collections
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

METRIC = "local energies/s + SR steps/s, 10×10 TFIM, BF16 vs FP64; p99 step latency"
PEAK = {  # MI355X dense peaks
    "mfma_fp64": 78.6e12, "mfma_fp32": 157.3e12, "mfma_bf16": 2.5e15,
    "valu_fp64": 78.6e12, "valu_fp32": 157.3e12, "hbm": 8.0e12,
}


def kernel_work(cls: str, w, precision: str):
    """Algorithmic work of one launch of a kernel class: (bound, flops or bytes, unit, peak).

    The two QGT contractions each apply J [Ns x P] (or its transpose) once:
    2 Ns P flops, over the factors of J, which are read once per launch:
    per sample the N spins (one bit each in the BF16/FP32 forms), M
    activations (8 B FP64; 4 B FP32 in the BF16/FP32 forms) and one 8-byte
    weight (w or z), plus one pass over a P-vector (4 B).  FP64
    runs on the FP64 matrix cores (78.6 TFLOP/s; 23 flop/B, above the 9.8 of
    the HBM ridge: MFMA-bound); the BF16 form (44 flop/B against a ridge of
    312) is HBM-bound.
    """
    N, M, Ns, C, K = w.n_sites, w.n_hidden, w.n_samples, w.n_chains, w.sweep_size
    P = N + M + N * M
    vf = "valu_fp64" if precision == "fp64" else "valu_fp32"
    if cls in ("outer", "qgt_w"):
        if precision == "fp64":
            return "mfma", 2.0 * Ns * P, "TFLOP/s", PEAK["mfma_fp64"]
        return "hbm", float(Ns * (N / 8.0 + 4 * M + 8) + 4 * P), "GB/s", PEAK["hbm"]
    if cls == "sample":
        # every proposal: M factors (FMA + MUL) of the amplitude ratio
        return "alu", 4.0 * C * K * M, "TFLOP/s", PEAK[vf]
    if cls == "eloc":
        # every sample: N single-flip ratios of M factors (MUL, FMA, MUL)
        return "alu", 6.0 * Ns * N * M / 2.0, "TFLOP/s", PEAK[vf]
    if cls == "theta":
        return "mfma", 2.0 * C * (N + 1) * M, "TFLOP/s", \
            PEAK["mfma_fp64" if precision == "fp64" else "mfma_bf16"]
    return "hbm", float("nan"), "GB/s", PEAK["hbm"]


# kernel class -> (source file of its kernel, symbol prefix in profiles)
KERNELS = {  # (BF16 form, the benchmark's main run)
    "qgt_w": ("qgt.hip", "k_w6"), "outer": ("qgt.hip", "k_outer7"),
    "reduce": ("qgt.hip", "k_update4<float>"),
    "sample": ("sampler.hip", "k_sample<float"), "eloc": ("eloc.hip", "k_eloc<float"),
    "theta": ("theta.hip", "k_theta_bf16"),
}
CSRC = os.path.join(ROOT, "paper_2112_10526_amd", "csrc")
PROFILES = os.path.join(ROOT, "profiles")


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
    """Markdown table of the wave-state counters (SQ_*) of the BF16 hot-path kernels."""
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
    for name in ["nqs::k_w6", "nqs::k_outer7", "nqs::k_update4<float>",
                 "nqs::k_sample<float, 4, 0, 2>", "nqs::k_sample<float, 16, 1, 1>",
                 "nqs::k_eloc<float, 0>", "nqs::k_eloc<float, 1>", "nqs::k_theta_bf16"]:
        if name not in agg:
            continue
        d = agg[name]
        wc = np.array(d["SQ_WAVE_CYCLES"])
        keep = wc >= 0.1 * wc.max()
        med = {k: float(np.median(np.array(v)[keep])) for k, v in d.items() if len(v) == len(wc)}
        w = med["SQ_WAVE_CYCLES"]
        out.append(f"| `{name}` | {med['SQ_WAVES']:.0f} | {w / med['SQ_WAVES']:.0f} | "
                   f"{100 * med['SQ_WAIT_ANY'] / w:.0f} | {100 * med['SQ_WAIT_INST_ANY'] / w:.0f} | "
                   f"{100 * med['SQ_ACTIVE_INST_ANY'] / w:.0f} |")
    print("\n".join(out))


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
    print("\n".join(out))


def make(w, precision):
    from paper_2112_10526_amd.nqs import VMCState
    st = VMCState.from_workload(w, precision=precision)
    st.thermalize(w.thermalize_segments)
    return st


def copy_rate_gbps(torch, mib=512, reps=10):
    """Measured HBM rate of a plain device copy (torch elementwise multiply by 1: one read
    and one write of a mib-MiB buffer), in GB/s of read + write bytes: context for the
    roofline fractions, which are taken against the published 8 TB/s."""
    n = mib * 2 ** 20 // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.mul(src, 1.0, out=dst)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.mul(src, 1.0, out=dst)
    e1.record()
    torch.cuda.synchronize()
    rate = 2.0 * n * 4 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    return rate


def stage_rooflines(w, precision, prof):
    """Each stage's kernel against its own binding roof (VALU for sampling and local
    energies, MFMA for theta and the FP64 contractions, HBM for the BF16 ones), from the
    event-timed warm-up launches: algorithmic work per launch / average launch time."""
    out = {}
    for cls in ("sample", "theta", "eloc", "qgt_w", "outer", "reduce"):
        p = prof.get(cls)
        if not p or not p["launches"]:
            continue
        bound, work, unit, peak = kernel_work(cls, w, precision)
        if not np.isfinite(work):
            continue
        us = p["ms"] * 1e3 / p["launches"]
        per_s = work / (us * 1e-6)
        scale = 1e12 if unit == "TFLOP/s" else 1e9
        out[cls] = dict(bound=bound, achieved=per_s / scale, peak=peak / scale, unit=unit,
                        frac=per_s / peak, avg_launch_us=us, launches=p["launches"])
    return out


def run_precision(w, precision, steps, warmup, torch):
    st = make(w, precision)
    # warm-up steps, profiled in full to find the dominant kernel class
    st.profile_enable(None)
    for _ in range(warmup):
        st.vmc_step(diag_shift=w.diag_shift, lr=w.lr, tol=w.cg_tol)
    prof = st.profile_read()
    dominant = max(prof, key=lambda k: prof[k]["ms"])
    # timed region: no event timing, CG batches replayed from graphs
    st.profile_enable([])
    lat, iters, acc, energies = [], [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        a = time.perf_counter()
        rep = st.vmc_step(diag_shift=w.diag_shift, lr=w.lr, tol=w.cg_tol)
        lat.append(time.perf_counter() - a)
        iters.append(rep.sr.iterations)
        acc.append(rep.energy["acceptance"])
        energies.append(rep.energy["mean"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # the same number of steps again with every launch of the dominant kernel
    # class bracketed by HIP events on its stream (launched one by one)
    st.profile_enable([dominant])
    torch.cuda.synchronize()
    e0 = time.perf_counter()
    iters_b = []
    for _ in range(steps):
        rep = st.vmc_step(diag_shift=w.diag_shift, lr=w.lr, tol=w.cg_tol)
        iters_b.append(rep.sr.iterations)
    torch.cuda.synchronize()
    e1 = time.perf_counter()
    tp = st.profile_read()[dominant]
    # stage rate: sampling + local energies, from a separately profiled step
    st.profile_enable(["sample", "theta", "eloc"])
    st.vmc_step(diag_shift=w.diag_shift, lr=w.lr, tol=w.cg_tol)
    sp = st.profile_read()
    stage_ms = sp["sample"]["ms"] + sp["theta"]["ms"] + sp["eloc"]["ms"]
    elapsed = t1 - t0
    lat_ms = np.array(lat) * 1e3
    out = dict(
        precision=precision,
        value=w.n_samples * steps / elapsed,
        ms_per_step=elapsed / steps * 1e3,
        sr_steps_per_s=steps / elapsed,
        p50_ms=float(np.percentile(lat_ms, 50)),
        p99_ms=float(np.percentile(lat_ms, 99)),
        cg_iters_mean=float(np.mean(iters)),
        acceptance_mean=float(np.mean(acc)),
        energy_first=energies[0], energy_last=energies[-1],
        stage_local_energies_per_s=w.n_samples / (stage_ms * 1e-3) if stage_ms > 0 else None,
        warmup_profile_ms={k: round(v["ms"] / max(warmup, 1), 4) for k, v in prof.items()
                           if v["launches"]},
        dominant=dict(kernel_class=dominant, launches=tp["launches"], total_ms=tp["ms"],
                      timed_pass_ms_per_step=(e1 - e0) / steps * 1e3,
                      timed_pass_cg_iters_mean=float(np.mean(iters_b))),
        stages=stage_rooflines(w, precision, prof),
    )
    st.close()
    return out


def dense_qgt_measure(torch, precision="fp32", repeats=2):
    """Dense Jacobian QGT at the N = 64 Heisenberg chain size (alpha = 8, 33,344
    parameters, 16,384 samples, FP32 matrices): one SR solve, each dense kernel
    event-timed and set against its own roof with its algorithmic work per launch:
      Jacobian build + centring: N_s P 4 bytes written (the matrix once; HBM),
      Gram matrix: N_s P (P + 1) flops (the symmetric product) on the FP32 matrix
        cores; in the BF16 form three BF16 products per FP32 product (hi hi + hi lo
        + lo hi), 3 N_s P (P + 1) flops on the BF16 matrix cores,
      dense product: P^2 4 bytes read (the matrix once; HBM)."""
    from paper_2112_10526_amd.nqs import VMCState
    w = synth.WORKLOADS["heis1d_n64"]
    st = VMCState.from_workload(w, precision=precision, qgt="jacobian_dense")
    s = torch.from_numpy(synth.sz0_configs(w.n_samples, w.n_sites, 12))
    P, Ns = w.n_params, w.n_samples
    gram = (("mfma", 3.0 * Ns * P * (P + 1.0), "TFLOP/s", PEAK["mfma_bf16"])
            if precision == "bf16" else ("mfma", Ns * P * (P + 1.0), "TFLOP/s", PEAK["mfma_fp32"]))
    work = {"jacobian": ("hbm", Ns * P * 4.0, "GB/s", PEAK["hbm"]),
            "gram": gram,
            "dense_matvec": ("hbm", P * P * 4.0, "GB/s", PEAK["hbm"])}
    best = {}
    for _ in range(repeats):
        st.load_samples(s)  # (a solve marks the batch and its gradient as used)
        st.expect_and_grad()
        st.profile_enable(list(work))
        t0 = time.perf_counter()
        _, info = st.sr_update(qgt="jacobian_dense", diag_shift=w.diag_shift, lr=0.0,
                               tol=w.cg_tol, maxiter=3000)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        prof = st.profile_read()
        for cls, (bound, wk, unit, peak) in work.items():
            p = prof[cls]
            # the product runs once per CG iteration; launches queued after the solve
            # has stopped return at once and are not counted
            n = min(p["launches"], info.iterations) if cls == "dense_matvec" else p["launches"]
            us = p["ms"] * 1e3 / max(n, 1)
            per_s = wk / (us * 1e-6)
            scale = 1e12 if unit == "TFLOP/s" else 1e9
            r = dict(bound=bound, achieved=per_s / scale, peak=peak / scale, unit=unit,
                     frac=per_s / peak, avg_launch_us=us, launches=n)
            if cls not in best or r["avg_launch_us"] < best[cls]["avg_launch_us"]:
                best[cls] = r
    st.close()
    return dict(metric="dense QGT kernels (N=64 Heisenberg chain, alpha=8, 16,384 samples)",
                workload="heis1d_n64: 1D Heisenberg N=64 periodic, Marshall, real RBM alpha=8, "
                         "33,344 parameters, FP32 Jacobian and Gram, FP64 CG",
                precision=precision, gram_matrix_cores="bf16 split" if precision == "bf16"
                else precision,
                n_params=P, n_samples=Ns, cg_iterations=info.iterations,
                solve_wall_ms=wall * 1e3, kernels=best, data="synthetic")


def precision_form_measure(torch, steps=5, warmup=1):
    """Precision form on the 16 x 16 Heisenberg workload (J1 = 1, periodic, Marshall
    rotated, zero magnetisation, exchange moves; alpha = 4, 1024 hidden units,
    263,424 parameters; 16,384 chains x 1 sample, 256 proposals between samples).
    The BF16 form (BF16 theta on the matrix cores with FP32 accumulation, FP32
    sampler and local energies, FP64 means and CG reductions) and the FP64 path run
    full SR steps from the same parameters and chains; then, on one sample batch
    drawn by the FP64 path, both evaluate local energies, energy statistics and the
    force from identical parameters, and the BF16 form's error against FP64 is
    reported (per-sample local energies, batch mean, force)."""
    w = synth.WORKLOADS["heis2d_l16"]
    runs, states = {}, {}
    for prec in ("bf16", "fp64"):
        st = make(w, prec)
        for _ in range(warmup):
            st.vmc_step(diag_shift=w.diag_shift, lr=w.lr, tol=w.cg_tol)
        lat, iters, acc = [], [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            a = time.perf_counter()
            rep = st.vmc_step(diag_shift=w.diag_shift, lr=w.lr, tol=w.cg_tol)
            lat.append(time.perf_counter() - a)
            iters.append(rep.sr.iterations)
            acc.append(rep.energy["acceptance"])
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        # sampling + local energies alone, event-timed in one more step
        st.profile_enable(["sample", "theta", "eloc"])
        st.vmc_step(diag_shift=w.diag_shift, lr=w.lr, tol=w.cg_tol)
        sp = st.profile_read()
        st.profile_enable([])
        stage_ms = sp["sample"]["ms"] + sp["theta"]["ms"] + sp["eloc"]["ms"]
        lat_ms = np.array(lat) * 1e3
        runs[prec] = dict(value=w.n_samples * steps / el, ms_per_step=el / steps * 1e3,
                          p50_ms=float(np.percentile(lat_ms, 50)),
                          p99_ms=float(np.percentile(lat_ms, 99)),
                          cg_iters_mean=float(np.mean(iters)),
                          acceptance_mean=float(np.mean(acc)),
                          stage_local_energies_per_s=w.n_samples / (stage_ms * 1e-3),
                          stage_ms={k: round(sp[k]["ms"], 4) for k in ("sample", "theta", "eloc")})
        states[prec] = st
        print(f"[bench] precision form {prec}: {runs[prec]['ms_per_step']:.2f} ms/step",
              file=sys.stderr, flush=True)
    # identical batch and parameters: the FP64 path's samples, its parameters
    ref, low = states["fp64"], states["bf16"]
    low.set_params(ref.get_params())
    s, _, _ = ref.sample()
    s = s.reshape(-1, w.n_sites)
    e64 = ref.local_energy(s).cpu().numpy()
    e16 = low.local_energy(s).cpu().numpy()
    ref.load_samples(s)
    low.load_samples(s)
    st64, g64 = ref.expect_and_grad()
    st16, g16 = low.expect_and_grad()
    g64, g16 = g64.cpu().numpy(), g16.cpu().numpy()
    err = dict(
        n_samples=int(e64.size),
        local_energy_max_rel=float(np.max(np.abs(e16 - e64) / np.maximum(np.abs(e64), 1.0))),
        mean_energy_fp64=st64["mean"], mean_energy_bf16=st16["mean"],
        mean_energy_rel=abs(st16["mean"] - st64["mean"]) / abs(st64["mean"]),
        error_of_mean_fp64=st64["error"],
        force_max_abs_err_rel_to_max=float(np.max(np.abs(g16 - g64)) / np.max(np.abs(g64))),
    )
    for st in states.values():
        st.close()
    return dict(metric="local energies/s, BF16 form vs FP64 path; energy error of the BF16 "
                       "form on an identical batch",
                workload="heis2d_l16: 2D Heisenberg J1 16x16 periodic, Marshall rotated, Sz=0, "
                         "exchange moves, real RBM alpha=4 (1024 hidden, 263,424 parameters), "
                         "16384 chains x 1 sample, 256 proposals per sample, SR on-the-fly QGT "
                         "+ CG tol 1e-6 shift 0.01 lr 0.01",
                unit="local energies/s", steps=steps, warmup=warmup, bf16=runs["bf16"],
                fp64=runs["fp64"], speedup=runs["bf16"]["value"] / runs["fp64"]["value"],
                energy_error_bf16_vs_fp64=err, data="synthetic")


def serve_measure(torch, n_runs=256, n_steps=10, loads=(0.5, 0.9, 1.5, 3.0), seed=7,
                  budget_gib=32, slots=32):
    """Serving form: a seeded stream of VMC runs (2D TFIM L x L, L ~ U{4..20},
    h ~ U[0.5, 4], alpha in {1, 2, 4}, 1024..16384 samples per step, BF16 form,
    n_steps SR steps each) through the continuous-batching server.

    Passes: (1) one run at a time, all present at the start (the single-run
    service rate mu = runs / wall); (2) all present at the start, up to `slots`
    resident, in lock-step ticks (every resident run advances one SR step per
    tick; a step's latency is its tick's) and with asynchronous steps (each run
    starts its next step when its previous one ends; a step's latency is its
    own); (3) Poisson arrivals at offered loads rho * mu, served in real time in
    lock-step ticks.  Each pass reports aggregate local energies/s, p50/p99
    SR-step latency, queueing delay, time in system, mean residency and peak HBM
    footprint."""
    from paper_2112_10526_amd.serving import Server, requests_from_stream
    budget = budget_gib << 30

    def summary(out):
        keys = ("wall_s", "ticks", "local_energies_per_s", "local_energies_per_busy_s",
                "mean_resident", "sr_steps", "p50_step_ms", "p99_step_ms",
                "queue_delay_ms_p50", "queue_delay_ms_p99", "run_latency_ms_p50",
                "run_latency_ms_p99", "peak_hbm_bytes")
        r = {k: out[k] for k in keys}
        r["errors"] = sum(1 for x in out["results"].values() if x.error)
        return r

    import dataclasses
    # (passes 1 and 2: every request present at time 0)
    base = [dataclasses.replace(r, arrival=0.0)
            for r in requests_from_stream(n_runs, seed, 1.0, n_steps=n_steps)]
    passes = {}
    last = [time.perf_counter()]

    def progress(done, total, steps):  # a line every 20 s during long passes
        now = time.perf_counter()
        if now - last[0] >= 20.0:
            last[0] = now
            print(f"[bench] serving: {done}/{total} runs finished, {steps} SR steps",
                  file=sys.stderr, flush=True)
    serial = Server(budget, max_slots=1).serve(base, realtime=False, progress=progress)
    passes["one_at_a_time"] = summary(serial)
    print(f"[bench] serving one at a time: {serial['wall_s']:.2f} s", file=sys.stderr, flush=True)
    mu = n_runs / serial["wall_s"]
    for mode in ("tick", "async"):
        cap = Server(budget, max_slots=slots, mode=mode).serve(base, realtime=False,
                                                               progress=progress)
        passes[f"all_present_{mode}"] = summary(cap)
        print(f"[bench] serving all present, {mode}: {cap['wall_s']:.2f} s", file=sys.stderr,
              flush=True)
    for rho in loads:
        reqs = requests_from_stream(n_runs, seed, rho * mu, n_steps=n_steps)
        out = Server(budget, max_slots=slots).serve(reqs, realtime=True, progress=progress)
        passes[f"poisson_rho_{rho}"] = dict(summary(out), offered_rate_runs_per_s=rho * mu)
        print(f"[bench] serving rho={rho}: {out['wall_s']:.2f} s", file=sys.stderr, flush=True)
    mix = collections.Counter((r.L, r.alpha) for r in base)
    return dict(metric="serving: aggregate local energies/s and p50/p99 SR-step latency",
                workload=(f"{n_runs} runs of 2D TFIM LxL, L~U{{4..20}}, h~U[0.5,4], alpha in "
                          f"{{1,2,4}}, 1024..16384 samples/step, {n_steps} SR steps each, BF16 "
                          f"form, stream seed {seed}"),
                unit="local energies/s", max_slots=slots, hbm_budget_bytes=budget,
                single_run_service_rate_runs_per_s=mu,
                total_local_energies=int(sum(r.n_samples * r.n_steps for r in base)),
                distinct_shapes=len(mix), passes=passes, data="synthetic")


def plain_measure(torch, steps=300, lr=0.05):
    """The small plain workload: periodic TFIM chain N = 10, J = h = 1, RBM alpha = 1,
    16 chains x 64 samples, 10 proposals between samples, SR shift 0.01.  SR steps
    from the N(0, 0.01^2) start (learning rate 0.05), timed one by one; the energy of
    the last 20 steps is set against the exact ground energy of the periodic chain,
    E0 = -(2 / sin(pi / 2N)) for J = h = 1 (free-fermion closed form).  At 1024 samples
    a step is launch-bound, so no roofline figure is given."""
    from paper_2112_10526_amd.nqs import VMCState
    w = synth.WORKLOADS["tfim1d_n10"]
    e0 = -2.0 / np.sin(np.pi / (2 * w.n_sites))
    out = {}
    for prec in ("fp64", "bf16"):
        st = VMCState.from_workload(w, precision=prec)
        st.thermalize(w.thermalize_segments)
        lat, energies, iters = [], [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            a = time.perf_counter()
            rep = st.vmc_step(diag_shift=w.diag_shift, lr=lr, tol=w.cg_tol)
            lat.append(time.perf_counter() - a)
            energies.append(rep.energy["mean"])
            iters.append(rep.sr.iterations)
        el = time.perf_counter() - t0
        st.close()
        e_last = float(np.mean(energies[-20:]))
        lat_ms = np.array(lat) * 1e3
        out[prec] = dict(ms_per_step=el / steps * 1e3, local_energies_per_s=w.n_samples * steps / el,
                         p50_ms=float(np.percentile(lat_ms, 50)),
                         p99_ms=float(np.percentile(lat_ms, 99)),
                         cg_iters_mean=float(np.mean(iters)), energy_first=energies[0],
                         energy_last20=e_last, rel_error_vs_exact=abs(e_last - e0) / abs(e0))
        print(f"[bench] plain {prec}: {out[prec]['ms_per_step']:.2f} ms/step, E = {e_last:.5f}",
              file=sys.stderr, flush=True)
    return dict(metric="SR steps on the N=10 TFIM chain: time per step and energy against the "
                       "exact ground energy",
                workload="tfim1d_n10: 1D TFIM N=10 periodic J=h=1, real RBM alpha=1 (120 "
                         "parameters), 16 chains x 64 samples, 10 proposals per sample, SR CG "
                         f"tol 1e-6 shift 0.01 lr {lr}",
                steps=steps, exact_ground_energy=e0, runs=out, data="synthetic")


def paper_workload_measure(torch, steps=10, warmup=2):
    """The workload closest to the one timed in the paper's comparison with jVMC (1D
    TFIM, L = 64, J = h = 1, periodic; RBM alpha = 1; 2^14 samples from 2^10 chains;
    dense Jacobian QGT with CG), with this library's real RBM (4,224 real parameters,
    where the paper's is complex) and 64 proposals between samples: full SR steps
    (sampling, local energies, gradient, QGT solve, update) with the dense and the
    on-the-fly QGT, FP64 path and BF16 form.  Context only: the model, precision and
    solver settings differ from the paper's."""
    from paper_2112_10526_amd.nqs import VMCState
    w = synth.Workload("tfim1d_n64", "tfim", "chain", 64, 1.0, 1.0, 1, 1024, 16, 64, "local",
                       "fp64")
    runs = {}
    for prec in ("fp64", "bf16"):
        for qgt in ("jacobian_dense", "onthefly"):
            st = VMCState.from_workload(w, precision=prec, qgt=qgt)
            st.thermalize(w.thermalize_segments)
            for _ in range(warmup):
                st.vmc_step(qgt=qgt, diag_shift=w.diag_shift, lr=w.lr, tol=w.cg_tol)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            iters = []
            for _ in range(steps):
                rep = st.vmc_step(qgt=qgt, diag_shift=w.diag_shift, lr=w.lr, tol=w.cg_tol)
                iters.append(rep.sr.iterations)
            torch.cuda.synchronize()
            el = (time.perf_counter() - t0) / steps
            runs[f"{prec}_{qgt}"] = dict(s_per_step=el, local_energies_per_s=w.n_samples / el,
                                         cg_iters_mean=float(np.mean(iters)))
            st.close()
            print(f"[bench] paper workload {prec} {qgt}: {el * 1e3:.2f} ms/step", file=sys.stderr,
                  flush=True)
    return dict(metric="seconds per VMC step, workload closest to the paper's timed one",
                workload="tfim1d_n64: 1D TFIM L=64 periodic J=h=1, real RBM alpha=1 (4,224 "
                         "parameters), 1024 chains x 16 samples, 64 proposals per sample, SR CG "
                         "tol 1e-6 shift 0.01",
                steps=steps, warmup=warmup, runs=runs,
                paper_context=dict(s_per_step=3.9, hardware="1x NVIDIA RTX 3090",
                                   model="complex RBM alpha=1, QGTJacobianDense(holomorphic) + CG",
                                   local_energies_per_s=16384 / 3.9),
                data="synthetic")


def cpu_baseline(w, n_chains=256, steps=2):
    """The oracle (plain FP64 CPU code) on a bounded sample of the workload:
    the first `n_chains` chains, one full SR step each time."""
    from oracle import core
    rbm = core.Rbm(w.n_sites, w.n_hidden, w.params())
    ham = core.Hamiltonian.tfim(w.n_sites, w.bonds(), w.J, w.h)
    ch = core.init_chains(w.n_sites, n_chains, w.chain_seed)
    th = core.sample(rbm, ch, 1, 10 * w.sweep_size, w.chain_seed, 0, mode="cached")
    ch, prop = th.chains, 10 * w.sweep_size
    times = []
    for _ in range(steps):
        t0 = time.perf_counter()
        rbm, ch, rep = core.vmc_step(rbm, ham, ch, w.samples_per_chain, w.sweep_size,
                                     w.chain_seed, prop, "local", w.diag_shift, w.lr, w.cg_tol)
        times.append(time.perf_counter() - t0)
        prop += w.samples_per_chain * w.sweep_size
    n = n_chains * w.samples_per_chain
    return dict(value=n / float(np.median(times)), unit="local energies/s",
                cores=core.num_threads(), kind="oracle",
                sample=(f"{n_chains} of 4096 chains x {w.samples_per_chain} samples "
                        f"({n} local energies) of the same 10x10 workload, full SR step "
                        f"(sampling, local energies, Jacobian, force, CG), median of {steps}"),
                seconds_per_step=float(np.median(times)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", default="bf16", choices=["bf16", "fp32", "fp64"])
    ap.add_argument("--compare", default="fp64", help="second precision to time ('' = none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--dense-qgt", action="store_true",
                    help="measure the dense Jacobian QGT kernels at the N=64 chain size instead")
    ap.add_argument("--precision-form", action="store_true",
                    help="measure the BF16 form against FP64 on the 16x16 Heisenberg workload")
    ap.add_argument("--plain", action="store_true",
                    help="SR steps on the N=10 TFIM chain: time and energy against the exact one")
    ap.add_argument("--paper-workload", action="store_true",
                    help="time full SR steps on the workload closest to the paper's timed one")
    ap.add_argument("--serve", action="store_true",
                    help="measure the continuous-batching server on a Poisson stream of runs")
    ap.add_argument("--serve-runs", type=int, default=256)
    ap.add_argument("--serve-steps", type=int, default=10)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run a plain device copy of this size first (counter calibration)")
    ap.add_argument("--summarize-stats", nargs=3, metavar=("CSV", "CMD", "TITLE"),
                    help="print a markdown table of a rocprofv3 kernel_stats.csv and exit")
    ap.add_argument("--summarize-mfma", nargs=3, metavar=("COUNTER_DIR", "CMD", "TITLE"),
                    help="print a markdown table of matrix-core counters and exit")
    ap.add_argument("--summarize-waves", nargs="+", metavar="COUNTER_DIR CMD [TITLE]",
                    help="print a markdown table of SQ wave-state counters and exit")
    ap.add_argument("--summarize-traffic", nargs=6,
                    metavar=("FETCH_DIR", "WRITE_DIR", "CLASS", "COPY_MIB", "FETCH_CMD", "WRITE_CMD"),
                    help="write profiles/traffic_*.md from two counter runs and exit")
    args = ap.parse_args()
    if args.summarize_stats:
        summarize_stats(*args.summarize_stats)
        return
    if args.summarize_mfma:
        summarize_mfma(*args.summarize_mfma)
        return
    if args.summarize_waves:
        summarize_waves(*args.summarize_waves)
        return
    if args.summarize_traffic:
        fd, wd, cls, mib, c1, c2 = args.summarize_traffic
        summarize_traffic(fd, wd, cls, args.precision, int(mib), (c1, c2))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); this library has "
              "no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.dense_qgt:
        for prec in ("fp32", "bf16"):
            print(json.dumps(dense_qgt_measure(torch, prec)), flush=True)
        return
    if args.precision_form:
        print(json.dumps(precision_form_measure(torch)), flush=True)
        return
    if args.serve:
        print(json.dumps(serve_measure(torch, args.serve_runs, args.serve_steps)), flush=True)
        return
    if args.paper_workload:
        print(json.dumps(paper_workload_measure(torch)), flush=True)
        return
    if args.plain:
        print(json.dumps(plain_measure(torch)), flush=True)
        return
    w = synth.WORKLOADS["tfim2d_l10"]
    if args.copy_probe_mib:
        n = args.copy_probe_mib * 2 ** 20 // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)  # one read + one write of the buffer
        torch.cuda.synchronize()
        del src, dst
    main_run = run_precision(w, args.precision, args.steps, args.warmup, torch)
    print(f"[bench] {args.precision}: {main_run['value']:.4g} local energies/s", file=sys.stderr,
          flush=True)
    cmp_run = None
    if args.compare and args.compare != args.precision:
        cmp_run = run_precision(w, args.compare, args.steps, args.warmup, torch)
        print(f"[bench] {args.compare}: {cmp_run['value']:.4g} local energies/s", file=sys.stderr,
              flush=True)
    dom = main_run["dominant"]
    bound, work, unit, peak = kernel_work(dom["kernel_class"], w, args.precision)
    avg_s = dom["total_ms"] * 1e-3 / max(dom["launches"], 1)
    achieved = work / avg_s if avg_s > 0 else float("nan")
    scale = 1e12 if unit == "TFLOP/s" else 1e9
    roofline = dict(bound=bound, kernel=dom["kernel_class"], achieved=achieved / scale,
                    peak=peak / scale, unit=unit, frac=achieved / peak,
                    avg_launch_us=avg_s * 1e6, work_per_launch=work,
                    traffic=read_traffic(dom["kernel_class"], args.precision),
                    measured_copy_GBps=copy_rate_gbps(torch))
    cpu = None if args.no_cpu_baseline else cpu_baseline(w)
    line = dict(
        metric=METRIC, value=main_run["value"], unit="local energies/s", n_gpus=1,
        steps=args.steps, warmup=args.warmup, ms_per_step=main_run["ms_per_step"],
        higher_is_better=True, scaling="weak", vs_baseline=None, dtype=args.precision,
        data="synthetic",
        config=dict(workload="tfim2d_l10: 2D TFIM 10x10 periodic J=1 h=3.044, real RBM alpha=2 "
                             "(200 hidden), 4096 chains x 4 samples, 100 proposals per sample, "
                             "SR on-the-fly QGT + CG tol 1e-6 shift 0.01 lr 0.01",
                    n_samples=w.n_samples, n_params=w.n_params, parallelism="1 GPU"),
        sr_steps_per_s=main_run["sr_steps_per_s"], p50_ms=main_run["p50_ms"],
        p99_ms=main_run["p99_ms"],
        stage_local_energies_per_s=main_run["stage_local_energies_per_s"],
        cg_iters_mean=main_run["cg_iters_mean"], acceptance=main_run["acceptance_mean"],
        roofline=roofline, stage_roofline=main_run["stages"], cpu_baseline=cpu,
        compare=cmp_run, detail=main_run,
    )
    print(json.dumps(line))


if __name__ == "__main__":
    main()
