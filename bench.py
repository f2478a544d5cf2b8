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
import ctypes
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


MEASURED = {}  # rates measured on the device by nqs_probe_rate (filled by measured_peaks)


def measured_peaks(torch) -> dict:
    """Rates of the instruction kinds the stages are bound by, measured on this
    device (nqs_probe_rate): flops/s for FMA and MFMA, exponentials/s for exp."""
    from paper_2112_10526_amd import _lib
    L = _lib.load()
    ctx = ctypes.c_void_p()
    if L.nqs_create(ctypes.byref(ctx), 0,
                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)):
        return {}
    out = {}
    for name, kind in _lib.PROBES.items():
        v = ctypes.c_double(0.0)
        if L.nqs_probe_rate(ctx, kind, ctypes.byref(v)) == 0:
            out[name] = v.value
    L.nqs_destroy(ctx)
    MEASURED.update(out)
    return out


def measured_peak(bound: str, cls: str, precision: str):
    """The measured counterpart of a roof (None where no probe covers it)."""
    if bound == "hbm":
        return MEASURED.get("copy_Bps")
    if bound == "mfma":
        if precision == "fp64":
            return MEASURED.get("fp64_mfma")
        return MEASURED.get("bf16_mfma") if (cls == "theta" and precision == "bf16") else None
    if bound == "alu":
        return MEASURED.get("fp64_fma" if precision == "fp64" else "fp32_fma")
    return None


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


from paper_2112_10526_amd.rocprof_summary import read_traffic  # noqa: E402


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
        mp = measured_peak(bound, cls, precision)
        out[cls] = dict(bound=bound, achieved=per_s / scale, peak=peak / scale, unit=unit,
                        frac=per_s / peak, avg_launch_us=us, launches=p["launches"],
                        measured_peak=None if mp is None else mp / scale,
                        frac_of_measured=None if mp is None else per_s / mp)
    return out


def trajectory(w, warmup, lat, iters, settle=20):
    """Where on the optimisation trajectory the timed steps lie.  The CG iteration
    count, and with it the step time, grows as the parameters move away from their
    start, so the rate is given for the timed steps within the first `settle` SR
    steps from the initial parameters ("init") and for those after them ("steady")."""
    idx = np.arange(len(lat)) + warmup + 1  # SR step number of each timed step
    out = dict(timed_sr_steps=[int(idx[0]), int(idx[-1])] if len(idx) else None,
               settle_steps=settle)
    for name, sel in (("init", idx <= settle), ("steady", idx > settle)):
        if sel.any():
            t = float(np.sum(np.asarray(lat)[sel]))
            out[name] = dict(steps=int(sel.sum()), local_energies_per_s=w.n_samples * sel.sum() / t,
                             ms_per_step=t / sel.sum() * 1e3,
                             cg_iters_mean=float(np.mean(np.asarray(iters)[sel])))
        else:
            out[name] = None
    return out


def run_precision(w, precision, steps, warmup, torch, step_log=None):
    st = make(w, precision)
    # warm-up steps, profiled in full to find the dominant kernel class
    st.profile_enable(None)
    for _ in range(warmup):
        st.vmc_step(diag_shift=w.diag_shift, lr=w.lr, tol=w.cg_tol)
    prof = st.profile_read()
    dominant = max(prof, key=lambda k: prof[k]["ms"])
    # timed region: no event timing, CG batches replayed from graphs
    st.profile_enable([])
    if step_log:
        st.open_step_log(step_log)
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
    if step_log:
        st.close_step_log()
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
        trajectory=trajectory(w, warmup, lat, iters),
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


def same_batch_cg_iters(torch, stages=4, steps_between=20):
    """CG iterations of the three forms on identical sample batches (10x10 TFIM):
    an FP64 trajectory advances steps_between SR steps per stage; at each stage
    its parameters and one freshly drawn batch are loaded into an FP64, an FP32
    and a BF16 state, and each solves the SR system on it (shift 0.01, tol 1e-6)."""
    from paper_2112_10526_amd.nqs import VMCState
    w = synth.WORKLOADS["tfim2d_l10"]
    ref = VMCState.from_workload(w, precision="fp64")
    rows = []
    for stage in range(stages):
        for _ in range(0 if stage == 0 else steps_between):
            ref.vmc_step(diag_shift=0.01, lr=0.01, tol=1e-6)
        p = ref.get_params()
        smp, _, _ = ref.sample()
        s = smp.reshape(-1, w.n_sites)
        row = dict(sr_steps=stage * steps_between)
        for prec in ("fp64", "fp32", "bf16"):
            st = VMCState.from_workload(w, precision=prec)
            st.set_params(p)
            st.load_samples(s)
            st.expect_and_grad()
            _, info = st.sr_update(diag_shift=0.01, lr=0.0, tol=1e-6, maxiter=4000)
            row[prec] = dict(iterations=info.iterations, converged=bool(info.converged))
            st.close()
        rows.append(row)
        print(f"[bench] same-batch CG iterations after {row['sr_steps']} steps: "
              + ", ".join(f"{k} {row[k]['iterations']}" for k in ("fp64", "fp32", "bf16")),
              file=sys.stderr, flush=True)
    ref.close()
    return dict(metric="CG iterations on identical sample batches, FP64 / FP32 / BF16 forms",
                workload="tfim2d_l10: 2D TFIM 10x10, alpha 2, 16,384 samples; SR shift 0.01, "
                         "CG tol 1e-6; parameters and samples from an FP64 trajectory",
                stages=rows, data="synthetic")


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
                  budget_gib=32, slots=32, only=None):
    """Serving form: a seeded stream of VMC runs (2D TFIM L x L, L ~ U{4..20},
    h ~ U[0.5, 4], alpha in {1, 2, 4}, 1024..16384 samples per step, BF16 form,
    n_steps SR steps each) through the continuous-batching server.

    Passes: (1) one run at a time, all present at the start (the single-run
    service rate mu = runs / wall); (2) all present at the start, up to `slots`
    resident, in lock-step ticks (every resident run advances one SR step per
    tick; a step's latency is its tick's) and with asynchronous steps (each run
    starts its next step when its previous one ends; a step's latency is its
    own), and in lock-step ticks with every run's CG iterations in its own
    launches instead of the grouped ones; the same two lock-step passes on
    n_runs / 2 small runs (L ~ U{4..8}, 1024..4096 samples); (3) Poisson
    arrivals at offered loads rho * mu, served in real time in lock-step
    ticks.  Each pass reports aggregate local energies/s, p50/p99
    SR-step latency, queueing delay, time in system, mean residency and peak HBM
    footprint.  only: names of the passes to run (all by default; the Poisson
    passes need the one-at-a-time pass, which then runs too)."""
    from paper_2112_10526_amd.serving import Server, requests_from_stream
    rho_names = [f"poisson_rho_{rho}" for rho in loads]

    def want(name):
        return only is None or name in only
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
    mu = None
    if want("one_at_a_time") or any(want(x) for x in rho_names):
        serial = Server(budget, max_slots=1).serve(base, realtime=False, progress=progress)
        passes["one_at_a_time"] = summary(serial)
        print(f"[bench] serving one at a time: {serial['wall_s']:.2f} s", file=sys.stderr,
              flush=True)
        mu = n_runs / serial["wall_s"]
    for mode in ("tick", "async"):
        if not want(f"all_present_{mode}"):
            continue
        cap = Server(budget, max_slots=slots, mode=mode).serve(base, realtime=False,
                                                               progress=progress)
        passes[f"all_present_{mode}"] = summary(cap)
        print(f"[bench] serving all present, {mode}: {cap['wall_s']:.2f} s", file=sys.stderr,
              flush=True)
    # lock-step ticks with every run's CG iterations in its own launches
    if want("all_present_tick_own_launches"):
        own = Server(budget, max_slots=slots, grouping=False).serve(base, realtime=False,
                                                                    progress=progress)
        passes["all_present_tick_own_launches"] = summary(own)
        print(f"[bench] serving all present, tick, own CG launches: {own['wall_s']:.2f} s",
              file=sys.stderr, flush=True)
    # small runs only (L 4..8, 1024..4096 samples, every one of them small enough
    # to group), grouped and in their own launches
    small = [dataclasses.replace(r, arrival=0.0)
             for r in requests_from_stream(n_runs // 2, seed, 1.0, n_steps=n_steps,
                                           L_range=(4, 8), samples=(1024, 2048, 4096))]
    for grouping in (True, False):
        key = "small_runs_tick" + ("" if grouping else "_own_launches")
        if not want(key):
            continue
        out = Server(budget, max_slots=slots, grouping=grouping).serve(small, realtime=False,
                                                                       progress=progress)
        passes[key] = summary(out)
        print(f"[bench] serving small runs, tick, grouping={grouping}: {out['wall_s']:.2f} s",
              file=sys.stderr, flush=True)
    for rho, name in zip(loads, rho_names):
        if not want(name):
            continue
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


def paper_workload_measure(torch, steps=5, warmup=2):
    """The workload timed in the paper's comparison with jVMC (table of VMC step
    times): 1D TFIM, L = 64, J = h = 1, periodic; complex RBM alpha = 1 with a
    holomorphic mapping (4,224 complex parameters); 2^14 samples from 2^10 chains
    (64 proposals between samples); the dense holomorphic QGT with CG.  Full SR
    steps: sampling, local energies, the embedded Jacobian, the force, the Gram
    matrix, CG and the update.  The Gram matrix is priced at the algorithmic
    4 N_s P^2 real flops of the Hermitian product dJ^H dJ (its upper triangle)."""
    from paper_2112_10526_amd.nqs import VMCState
    w = synth.WORKLOADS["tfim1d_n64_c"]
    direct = paper_workload_direct(torch, w, steps, warmup)
    st = VMCState.from_workload(w)
    st.thermalize(w.thermalize_segments)
    st.profile_enable(None)
    for _ in range(warmup):
        st.vmc_step(diag_shift=w.diag_shift, lr=w.lr, tol=w.cg_tol)
    prof = st.profile_read()
    st.profile_enable([])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters, energies = [], []
    for _ in range(steps):
        rep = st.vmc_step(diag_shift=w.diag_shift, lr=w.lr, tol=w.cg_tol)
        iters.append(rep.sr.iterations)
        energies.append(rep.energy["mean"])
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    st.close()
    P, Ns = w.n_params, w.n_samples
    g = prof["gram"]
    gram_us = g["ms"] * 1e3 / max(g["launches"], 1)
    gram_flops = 4.0 * Ns * P * P
    print(f"[bench] paper workload (complex): {el * 1e3:.2f} ms/step, Gram {gram_us:.0f} us",
          file=sys.stderr, flush=True)
    return dict(metric="seconds per VMC step on the paper's timed workload",
                value=el, unit="s/step", higher_is_better=False, steps=steps, warmup=warmup,
                dtype="c128", data="synthetic",
                config=dict(workload="tfim1d_n64_c: 1D TFIM L=64 periodic J=h=1, complex RBM "
                                     "alpha=1 (4,224 complex parameters), 1024 chains x 16 "
                                     "samples, 64 proposals per sample, dense holomorphic QGT "
                                     f"+ CG tol {w.cg_tol} shift {w.diag_shift} lr {w.lr}",
                            n_samples=Ns, n_params=P),
                local_energies_per_s=Ns / el, cg_iters_mean=float(np.mean(iters)),
                energy_first=energies[0], energy_last=energies[-1],
                warmup_profile_ms={k: round(v["ms"] / warmup, 4) for k, v in prof.items()
                                   if v["launches"]},
                gram=dict(bound="mfma", avg_launch_us=gram_us, algorithmic_flops=gram_flops,
                          achieved=gram_flops / (gram_us * 1e-6) / 1e12, peak=78.6,
                          unit="TFLOP/s", frac=gram_flops / (gram_us * 1e-6) / 78.6e12),
                direct_solve=direct,
                paper_context=dict(hardware="1x NVIDIA RTX 3090 (paper's table)",
                                   s_per_step_cg=3.9, s_per_step_svd=24.0,
                                   s_per_step_cg_2gpu=1.7))


def paper_workload_direct(torch, w, steps, warmup):
    """The same SR steps with the dense system solved directly (Cholesky of the
    real embedding, size 2P = 8448) instead of by CG: the counterpart of the
    paper's dense-solver row."""
    from paper_2112_10526_amd.nqs import VMCState
    st = VMCState(model=w.model, n_sites=w.n_sites, bonds=w.bonds(), J=w.J, h=w.h,
                  n_hidden=w.n_hidden, precision=w.precision, rule=w.rule,
                  n_chains=w.n_chains, samples_per_chain=w.samples_per_chain,
                  sweep_size=w.sweep_size, seed=w.chain_seed, params=w.params(),
                  dense_solver="cholesky")
    st.thermalize(w.thermalize_segments)
    st.profile_enable(None)
    for _ in range(warmup):
        st.vmc_step(diag_shift=w.diag_shift, lr=w.lr, tol=w.cg_tol)
    prof = st.profile_read()
    st.profile_enable([])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        st.vmc_step(diag_shift=w.diag_shift, lr=w.lr, tol=w.cg_tol)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    st.close()
    print(f"[bench] paper workload (complex, Cholesky): {el * 1e3:.2f} ms/step", file=sys.stderr,
          flush=True)
    return dict(s_per_step=el, warmup_profile_ms={k: round(v["ms"] / warmup, 4)
                                                  for k, v in prof.items() if v["launches"]})


def tdvp_quench_measure(torch, steps=100, dt=0.01, prep_steps=300, diag_shift=1e-3,
                        observe_every=10, solver="cholesky"):
    """The real-time example: TFIM chain L = 20 (J = 1), complex RBM alpha = 1,
    4096 samples.  The initial state is the h = 1/2 ground state found by SR
    (the example's 300 steps, learning rate 0.01, shift 0.01); the field is then
    quenched to h = 1 and the state evolved by TDVP Heun steps of dt up to
    t = steps dt with the dense holomorphic QGT and CG.  Reports the time per
    TDVP step (two evaluations of the equation of motion: sampling, local
    energies, Jacobian, force, Gram, CG) and the trace of the energy (conserved
    by the exact dynamics) and of sum_i <sigma^x_i> (local estimator
    sum_i psi(s^i)/psi(s) = (J sum_<ab> s_a s_b - E_loc(s)) / h, from a batch
    drawn after the step, outside the timed calls)."""
    from paper_2112_10526_amd.nqs import VMCState
    w = synth.WORKLOADS["tfim1d_n20_quench"]
    b = w.bonds()
    prep = VMCState.from_workload(w.replace(h=0.5))
    prep.thermalize(w.thermalize_segments)
    for _ in range(prep_steps):
        rep = prep.vmc_step(qgt="jacobian_dense", diag_shift=0.01, lr=0.01, tol=1e-6)
    e_prep = rep.energy["mean"]
    st = VMCState(model=w.model, n_sites=w.n_sites, bonds=b, J=w.J, h=w.h, n_hidden=w.n_hidden,
                  precision=w.precision, rule=w.rule, n_chains=w.n_chains,
                  samples_per_chain=w.samples_per_chain, sweep_size=w.sweep_size,
                  seed=w.chain_seed, params=prep.get_params(), dense_solver=solver)
    st.set_chains(prep.get_chains())
    prep.close()

    def observe(t):
        smp, _, _ = st.sample()
        s = smp.reshape(-1, w.n_sites)
        E = st.local_energy(s).cpu().numpy()
        sc = s.cpu().numpy().astype(np.float64)
        zz = (sc[:, b[:, 0]] * sc[:, b[:, 1]]).sum(axis=1)
        sx = (w.J * zz - E.real) / w.h
        n = sx.size
        return dict(t=t, energy=float(E.real.mean()), energy_err=float(E.real.std() / np.sqrt(n)),
                    sx=float(sx.mean()), sx_err=float(sx.std() / np.sqrt(n)))

    trace = [observe(0.0)]
    lat, iters = [], []
    for k in range(1, steps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stages = st.tdvp_step(dt, gamma=-1j, scheme="heun", diag_shift=diag_shift, tol=1e-6)
        lat.append(time.perf_counter() - t0)  # (the step reads its scalars back: synchronous)
        iters.append(np.mean([g["solve"].iterations for g in stages]))
        if k % observe_every == 0:
            trace.append(observe(k * dt))
    st.close()
    lat_ms = np.array(lat) * 1e3
    e = np.array([r["energy"] for r in trace])
    print(f"[bench] TDVP quench ({solver}): {np.median(lat_ms):.2f} ms per Heun step",
          file=sys.stderr, flush=True)
    return dict(metric="milliseconds per TDVP (Heun) step, quench of the TFIM chain",
                value=float(np.mean(lat_ms)), unit="ms/step", higher_is_better=False,
                p50_ms=float(np.percentile(lat_ms, 50)), p99_ms=float(np.percentile(lat_ms, 99)),
                steps=steps, dt=dt, dtype="c128", data="synthetic",
                config=dict(workload="tfim1d_n20_quench: 1D TFIM L=20 periodic J=1, h 0.5 -> 1, "
                                     "complex RBM alpha=1 (440 complex parameters), 256 chains "
                                     "x 16 samples, 20 proposals per sample, Heun dt "
                                     f"{dt}, dense holomorphic QGT solved by {solver} "
                                     f"(CG tol 1e-6), shift {diag_shift}",
                            n_samples=w.n_samples, n_params=w.n_params),
                prep=dict(sr_steps=prep_steps, energy_h05=e_prep),
                cg_iters_mean=float(np.mean(iters)),
                energy_drift=float(e.max() - e.min()),
                energy_err_mean=float(np.mean([r["energy_err"] for r in trace])),
                trace=trace)


def symm_measure(torch, steps=20, warmup=3):
    """Full SR steps of the translation-symmetric RBM on the 10x10 TFIM workload
    (alpha = 2 features over the 100 translations: the same 200 hidden units as
    the plain alpha = 2 RBM, but 203 parameters instead of 20,300), dense QGT +
    CG over the symmetric parameters, FP64 path and BF16 form."""
    from paper_2112_10526_amd.nqs import VMCState
    w = synth.WORKLOADS["tfim2d_l10"]
    perms = synth.square_translations(w.L)
    runs = {}
    for prec, solver in (("fp64", "cg"), ("bf16", "cg"), ("fp64", "cholesky"),
                         ("bf16", "cholesky")):
        st = VMCState(model="tfim", n_sites=w.n_sites, bonds=w.bonds(), J=w.J, h=w.h,
                      n_hidden=0, precision=prec, rule="local", n_chains=w.n_chains,
                      samples_per_chain=w.samples_per_chain, sweep_size=w.sweep_size,
                      seed=w.chain_seed, params=synth.symm_params(w.n_sites, 2, w.param_seed),
                      symmetries=perms, alpha=2, dense_solver=solver)
        st.thermalize(w.thermalize_segments)
        st.profile_enable(None)
        for _ in range(warmup):
            st.vmc_step(diag_shift=w.diag_shift, lr=w.lr, tol=w.cg_tol)
        prof = st.profile_read()
        st.profile_enable([])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        iters, energies = [], []
        for _ in range(steps):
            rep = st.vmc_step(diag_shift=w.diag_shift, lr=w.lr, tol=w.cg_tol)
            iters.append(rep.sr.iterations)
            energies.append(rep.energy["mean"])
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / steps
        runs[f"{prec}_{solver}"] = dict(ms_per_step=el * 1e3, local_energies_per_s=w.n_samples / el,
                          cg_iters_mean=float(np.mean(iters)), energy_first=energies[0],
                          energy_last=energies[-1],
                          warmup_profile_ms={k: round(v["ms"] / warmup, 4)
                                             for k, v in prof.items() if v["launches"]})
        st.close()
        print(f"[bench] symmetric RBM {prec} {solver}: {el * 1e3:.2f} ms/step", file=sys.stderr,
              flush=True)
    return dict(metric="SR steps of the translation-symmetric RBM", unit="ms/step",
                workload="tfim2d_l10 with RBMSymm: 2D TFIM 10x10 periodic J=1 h=3.044, alpha=2 "
                         "over 100 translations (203 parameters), 4096 chains x 4 samples, 100 "
                         "proposals per sample, dense QGT solved by CG (tol 1e-6) or Cholesky, "
                         "shift 0.01 lr 0.01",
                steps=steps, warmup=warmup, runs=runs, data="synthetic")


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(w, n_chains=1024, steps=5):
    """The oracle (plain FP64 CPU code, OpenMP over all host threads) on a bounded
    sample of the workload: the first `n_chains` of its chains (a quarter of the
    batch), thermalised, then one untimed warm-up SR step and `steps` timed full SR
    steps (sampling, local energies, Jacobian, force, CG solve, update); median and
    minimum of the timed steps, as the paper times its own runs."""
    from oracle import core
    rbm = core.Rbm(w.n_sites, w.n_hidden, w.params())
    ham = core.Hamiltonian.tfim(w.n_sites, w.bonds(), w.J, w.h)
    ch = core.init_chains(w.n_sites, n_chains, w.chain_seed)
    th = core.sample(rbm, ch, 1, 10 * w.sweep_size, w.chain_seed, 0, mode="cached")
    ch, prop = th.chains, 10 * w.sweep_size
    times, iters = [], []
    for k in range(steps + 1):
        t0 = time.perf_counter()
        rbm, ch, rep = core.vmc_step(rbm, ham, ch, w.samples_per_chain, w.sweep_size,
                                     w.chain_seed, prop, "local", w.diag_shift, w.lr, w.cg_tol)
        dt = time.perf_counter() - t0
        prop += w.samples_per_chain * w.sweep_size
        if k > 0:  # the first step is the warm-up
            times.append(dt)
            iters.append(rep.cg_iters)
    n = n_chains * w.samples_per_chain
    med, best = float(np.median(times)), float(np.min(times))
    return dict(value=n / med, unit="local energies/s", cores=core.num_threads(),
                kind="oracle", cpu_model=cpu_model(),
                sample=(f"{n_chains} of the {w.n_chains} chains x {w.samples_per_chain} samples "
                        f"({n} of the {w.n_samples} local energies per SR step) of the same "
                        f"10x10 workload; 1 warm-up and {steps} timed full SR steps (sampling, "
                        f"local energies, Jacobian, force, CG, update); value from the median "
                        f"step, the CG iteration count is that of the smaller batch"),
                seconds_per_step_median=med, seconds_per_step_min=best,
                value_from_min=n / best, cg_iters_mean=float(np.mean(iters)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", default="bf16", choices=["bf16", "fp32", "fp64"])
    ap.add_argument("--compare", default="fp64", help="second precision to time ('' = none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--step-log", default="",
                    help="append one JSON line per timed SR step of the main run to this file")
    ap.add_argument("--dense-qgt", action="store_true",
                    help="measure the dense Jacobian QGT kernels at the N=64 chain size instead")
    ap.add_argument("--precision-form", action="store_true",
                    help="measure the BF16 form against FP64 on the 16x16 Heisenberg workload")
    ap.add_argument("--same-batch-iters", action="store_true",
                    help="CG iterations of the FP64, FP32 and BF16 forms on identical batches")
    ap.add_argument("--plain", action="store_true",
                    help="SR steps on the N=10 TFIM chain: time and energy against the exact one")
    ap.add_argument("--paper-workload", action="store_true",
                    help="time full SR steps on the paper's timed workload (complex RBM)")
    ap.add_argument("--tdvp-quench", action="store_true",
                    help="time TDVP Heun steps of the L=20 TFIM quench (complex RBM)")
    ap.add_argument("--symm", action="store_true",
                    help="time SR steps of the translation-symmetric RBM (10x10 TFIM)")
    ap.add_argument("--serve", action="store_true",
                    help="measure the continuous-batching server on a Poisson stream of runs")
    ap.add_argument("--serve-runs", type=int, default=256)
    ap.add_argument("--serve-steps", type=int, default=10)
    ap.add_argument("--serve-passes", default="",
                    help="comma-separated serving passes to run (default: all)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run a plain device copy of this size first (counter calibration)")
    args = ap.parse_args()
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
    if args.same_batch_iters:
        print(json.dumps(same_batch_cg_iters(torch)), flush=True)
        return
    if args.serve:
        only = set(x for x in args.serve_passes.split(",") if x) or None
        print(json.dumps(serve_measure(torch, args.serve_runs, args.serve_steps, only=only)),
              flush=True)
        return
    if args.paper_workload:
        print(json.dumps(paper_workload_measure(torch)), flush=True)
        return
    if args.symm:
        print(json.dumps(symm_measure(torch)), flush=True)
        return
    if args.tdvp_quench:
        out = tdvp_quench_measure(torch, solver="cholesky")
        out["cg_run"] = {k: v for k, v in tdvp_quench_measure(torch, solver="cg").items()
                         if k in ("value", "p50_ms", "cg_iters_mean", "energy_drift")}
        print(json.dumps(out), flush=True)
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
    # the device's own ceilings (copy rate and instruction-kind probes), taken
    # before the runs so that every stage roofline can be set against them
    copy_gbps = copy_rate_gbps(torch)
    MEASURED["copy_Bps"] = copy_gbps * 1e9
    probes = measured_peaks(torch)
    main_run = run_precision(w, args.precision, args.steps, args.warmup, torch,
                             step_log=args.step_log or None)
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
                    measured_copy_GBps=copy_gbps)
    mp = measured_peak(bound, dom["kernel_class"], args.precision)
    roofline.update(measured_peak=None if mp is None else mp / scale,
                    frac_of_measured=None if mp is None else achieved / mp)
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
        trajectory=main_run["trajectory"],
        roofline=roofline, stage_roofline=main_run["stages"], cpu_baseline=cpu,
        measured_peaks=dict(copy_GBps=copy_gbps,
                            **{k + ("_Gexp_per_s" if k.endswith("exp") else "_TFLOPs"):
                               v / (1e9 if k.endswith("exp") else 1e12)
                               for k, v in probes.items()}),
        compare=cmp_run, detail=main_run,
    )
    print(json.dumps(line))


if __name__ == "__main__":
    main()
