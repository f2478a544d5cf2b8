"""Continuous-batching server for many concurrent VMC runs on one GPU.

Each request is one VMC run (2D TFIM L x L, field h, RBM density alpha,
samples per step, number of SR steps).  The server

  * admits requests in arrival order as soon as a slot is free and the run's
    HBM footprint (its exact workspace size, ``nqs_workspace_bytes``) fits in
    the remaining budget, so requests that arrive while others are running
    join at the next tick;
  * keeps every admitted run's chains, parameters and tables resident in its
    own device workspace until the run finishes, then frees it;
  * advances all resident runs by one SR step per tick with
    ``nqs_batch_step``, which issues every run's kernels on that run's own
    HIP stream in lock-step, so the runs' kernels overlap on the device.

Every run's arithmetic is independent of the others (its own Philox stream,
fixed-order reductions), so a run's trajectory in the mix is identical to the
same run served alone.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Callable, List, Optional

import numpy as np
import torch

import synth

from .nqs import VMCState, batch_step


@dataclasses.dataclass
class Request:
    id: int
    arrival: float          # seconds after the start of serving
    L: int
    h: float
    alpha: int
    n_samples: int
    n_steps: int
    param_seed: int = 1
    chain_seed: int = 2
    samples_per_chain: int = 4

    def workload(self, precision: str) -> synth.Workload:
        n_chains = max(1, self.n_samples // self.samples_per_chain)
        return synth.Workload(f"serve{self.id}", "tfim", "square", self.L, 1.0, self.h,
                              self.alpha, n_chains, self.samples_per_chain, self.L * self.L,
                              "local", precision, param_seed=self.param_seed,
                              chain_seed=self.chain_seed)


@dataclasses.dataclass
class RunResult:
    id: int
    arrival: float
    admitted: Optional[float] = None
    finished: Optional[float] = None
    footprint: int = 0
    energies: List[float] = dataclasses.field(default_factory=list)
    cg_iters: List[int] = dataclasses.field(default_factory=list)
    step_latency: List[float] = dataclasses.field(default_factory=list)
    params: Optional[np.ndarray] = None
    error: Optional[str] = None


class Server:
    def __init__(self, hbm_budget: int, max_slots: int = 64, n_streams: int = 4,
                 precision: str = "bf16", device: int = 0, thermalize_segments: int = 20,
                 diag_shift: float = 0.01, lr: float = 0.01, cg_tol: float = 1e-6,
                 keep_params: bool = False, state_factory=None, step_fn=None, streams=None):
        self.budget = int(hbm_budget)
        self.max_slots = max_slots
        self.precision = precision
        self.device = device
        self.therm = thermalize_segments
        self.cfg = dict(diag_shift=diag_shift, lr=lr, tol=cg_tol)
        if streams is None:
            streams = [torch.cuda.Stream(device=device) for _ in range(n_streams)]
        self.streams = streams
        self.keep_params = keep_params
        self.peak_used = 0
        self.make_state = state_factory or self._make_state
        self.step = step_fn or batch_step

    def _make_state(self, req: Request, stream):
        w = req.workload(self.precision)
        return VMCState.from_workload(w, stream=stream, device=self.device, allocate=False)

    def serve(self, requests: List[Request], clock: Callable[[], float] = time.perf_counter,
              realtime: bool = True) -> dict:
        """Serve every request; with realtime=False arrival times are ignored
        (all requests are present at the start)."""
        pending = sorted(requests, key=lambda r: (r.arrival, r.id))
        results = {r.id: RunResult(r.id, r.arrival) for r in requests}
        active = []  # (request, state, footprint, steps_done)
        used = 0
        t0 = clock()
        n_tick = 0
        resident = 0  # sum over ticks of the runs advanced in that tick
        busy = 0.0    # seconds spent inside ticks
        local_energies = 0
        while pending or active:
            now = clock() - t0
            # admission in arrival order
            while pending and len(active) < self.max_slots and (
                    not realtime or pending[0].arrival <= now):
                req = pending[0]
                stream = self.streams[req.id % len(self.streams)]
                st = self.make_state(req, stream)
                fp = st.workspace_bytes
                if fp > self.budget:
                    results[req.id].error = f"footprint {fp} B exceeds the budget {self.budget} B"
                    st.close()
                    pending.pop(0)
                    continue
                if used + fp > self.budget:
                    st.close()
                    break  # wait for memory to free up
                pending.pop(0)
                st.bind()
                st.thermalize(self.therm)
                used += fp
                self.peak_used = max(self.peak_used, used)
                res = results[req.id]
                res.admitted = clock() - t0
                res.footprint = fp
                active.append([req, st, fp, 0])
            if not active:
                if pending and realtime:
                    time.sleep(max(0.0, min(0.01, pending[0].arrival - (clock() - t0))))
                continue
            # one tick: one SR step for every resident run
            a = clock()
            reps = self.step([x[1] for x in active], [self.cfg] * len(active))
            dt = clock() - a
            n_tick += 1
            resident += len(active)
            busy += dt
            still = []
            for (req, st, fp, done), rep in zip(active, reps):
                res = results[req.id]
                res.energies.append(rep.energy["mean"])
                res.cg_iters.append(rep.sr.iterations)
                res.step_latency.append(dt)
                local_energies += st.n_samples
                done += 1
                if done >= req.n_steps:
                    if self.keep_params:
                        res.params = st.get_params()
                    st.close()
                    used -= fp
                    res.finished = clock() - t0
                else:
                    still.append([req, st, fp, done])
            active = still
        total = clock() - t0
        lat = np.array([x for r in results.values() for x in r.step_latency])
        done = [r for r in results.values() if r.admitted is not None]
        queue = np.array([(r.admitted - r.arrival) * 1e3 for r in done] or [0.0])
        in_sys = np.array([(r.finished - r.arrival) * 1e3 for r in done
                           if r.finished is not None] or [0.0])

        def pct(a, q):
            return float(np.percentile(a, q)) if a.size else None
        return dict(
            results=results, wall_s=total, ticks=n_tick,
            local_energies_per_s=local_energies / total if total > 0 else 0.0,
            local_energies_per_busy_s=local_energies / busy if busy > 0 else 0.0,
            mean_resident=resident / n_tick if n_tick else 0.0,
            sr_steps=int(lat.size),
            p50_step_ms=pct(lat * 1e3, 50), p99_step_ms=pct(lat * 1e3, 99),
            queue_delay_ms_p50=pct(queue, 50), queue_delay_ms_p99=pct(queue, 99),
            run_latency_ms_p50=pct(in_sys, 50), run_latency_ms_p99=pct(in_sys, 99),
            peak_hbm_bytes=self.peak_used,
        )


def requests_from_stream(n_runs: int, seed: int, rate: float, n_steps: int = 50, **kw) -> List[Request]:
    """Requests of a seeded Poisson stream (see ``synth.serve_stream``)."""
    out = []
    for d in synth.serve_stream(n_runs, seed, rate, n_steps=n_steps, **kw):
        out.append(Request(d["id"], d["arrival"], d["L"], d["h"], d["alpha"], d["n_samples"],
                           d["n_steps"], d["param_seed"], d["chain_seed"]))
    return out
