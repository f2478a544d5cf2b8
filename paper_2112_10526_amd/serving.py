"""Continuous-batching server for many concurrent VMC runs on one GPU.

Each request is one VMC run (2D TFIM L x L, field h, RBM density alpha,
samples per step, number of SR steps).  The server

  * admits requests in arrival order as soon as a slot is free and the run's
    HBM footprint (its exact workspace size, ``nqs_workspace_bytes``) fits in
    the remaining budget, so requests that arrive while others are running
    join at the next tick;
  * keeps every admitted run's chains, parameters and tables resident in its
    own device workspace until the run finishes, then frees it;
  * advances the resident runs on their own HIP streams, so the runs' kernels
    overlap on the device.  Default (mode "tick"): all resident runs advance by
    one SR step per tick with ``nqs_batch_step``, whose on-the-fly CG runs the
    iterations of all resident BF16/FP32-form runs as one launch per kernel
    class (``grouping``; off: each run launches its own); mode "async": every
    run starts its next SR step as soon as its previous one has finished
    (``nqs_step_begin`` / ``nqs_step_poll``), with no barrier between runs.

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

from .lattice import RunSpec
from .nqs import VMCState, batch_step, step_begin, step_poll


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

    def workload(self, precision: str) -> RunSpec:
        n_chains = max(1, self.n_samples // self.samples_per_chain)
        return RunSpec("tfim", "square", self.L, 1.0, self.h, self.alpha, n_chains,
                       self.samples_per_chain, self.L * self.L, "local", precision,
                       param_seed=self.param_seed, chain_seed=self.chain_seed)


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
                 keep_params: bool = False, state_factory=None, step_fn=None, streams=None,
                 mode: str = "tick", begin_fn=None, poll_fn=None, grouping: bool = True):
        if mode not in ("async", "tick"):
            raise ValueError(f"unknown serving mode {mode!r}")
        self.mode = mode
        self.grouping = grouping
        self.begin = begin_fn or step_begin
        self.poll = poll_fn or step_poll
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
              realtime: bool = True, progress: Optional[Callable[[int, int, int], None]] = None
              ) -> dict:
        """Serve every request; with realtime=False arrival times are ignored
        (all requests are present at the start).  progress, if given, is called
        after every tick with (runs finished, runs in total, SR steps done)."""
        pending = sorted(requests, key=lambda r: (r.arrival, r.id))
        results = {r.id: RunResult(r.id, r.arrival) for r in requests}
        active = []  # [request, state, footprint, steps done, step start or None]
        self._used = 0
        t0 = clock()
        n_tick = 0
        resident = 0  # sum over ticks (polls) of the runs resident
        busy = 0.0    # seconds spent inside ticks (polls)
        local_energies = 0
        while pending or active:
            self._admit(pending, active, results, clock, t0, realtime)
            if not active:
                if pending and realtime:
                    time.sleep(max(0.0, min(0.01, pending[0].arrival - (clock() - t0))))
                continue
            a = clock()
            if self.mode == "tick":
                # one tick: one SR step for every resident run
                reps = self.step([x[1] for x in active], [self.cfg] * len(active))
                t1 = clock()
                finished = [(x, rep, t1 - a) for x, rep in zip(active, reps)]
            else:
                # every idle run starts its next step; then wait for any to end
                for x in active:
                    if x[4] is None:
                        self.begin(x[1], self.cfg)
                        x[4] = clock()
                done = self.poll([x[1] for x in active], True)
                t1 = clock()
                finished = [(active[k], rep, t1 - active[k][4]) for k, rep in done.items()]
            n_tick += 1
            resident += len(active)
            busy += t1 - a
            for x, rep, dt in finished:
                req, st = x[0], x[1]
                res = results[req.id]
                res.energies.append(rep.energy["mean"])
                res.cg_iters.append(rep.sr.iterations)
                res.step_latency.append(dt)
                local_energies += st.n_samples
                x[3] += 1
                x[4] = None
                if x[3] >= req.n_steps:
                    if self.keep_params:
                        res.params = st.get_params()
                    st.close()
                    self._used -= x[2]
                    res.finished = clock() - t0
            active[:] = [x for x in active if x[3] < x[0].n_steps]
            if progress is not None:
                progress(sum(1 for r in results.values() if r.finished is not None),
                         len(requests), sum(len(r.energies) for r in results.values()))
        total = clock() - t0
        lat = np.array([x for r in results.values() for x in r.step_latency])
        done = [r for r in results.values() if r.admitted is not None]
        queue = np.array([(r.admitted - r.arrival) * 1e3 for r in done] or [0.0])
        in_sys = np.array([(r.finished - r.arrival) * 1e3 for r in done
                           if r.finished is not None] or [0.0])

        def pct(a, q):
            return float(np.percentile(a, q)) if a.size else None
        return dict(
            results=results, wall_s=total, ticks=n_tick, mode=self.mode,
            local_energies_per_s=local_energies / total if total > 0 else 0.0,
            local_energies_per_busy_s=local_energies / busy if busy > 0 else 0.0,
            mean_resident=resident / n_tick if n_tick else 0.0,
            sr_steps=int(lat.size),
            p50_step_ms=pct(lat * 1e3, 50), p99_step_ms=pct(lat * 1e3, 99),
            queue_delay_ms_p50=pct(queue, 50), queue_delay_ms_p99=pct(queue, 99),
            run_latency_ms_p50=pct(in_sys, 50), run_latency_ms_p99=pct(in_sys, 99),
            peak_hbm_bytes=self.peak_used,
        )

    def _admit(self, pending, active, results, clock, t0, realtime):
        """Admission in arrival order while a slot is free and the run's footprint
        fits in what is left of the budget."""
        now = clock() - t0
        while pending and len(active) < self.max_slots and (
                not realtime or pending[0].arrival <= now):
            req = pending[0]
            stream = self.streams[req.id % len(self.streams)]
            st = self.make_state(req, stream)
            if not self.grouping:
                st.set_cg_grouping(False)
            fp = st.workspace_bytes
            if fp > self.budget:
                results[req.id].error = f"footprint {fp} B exceeds the budget {self.budget} B"
                st.close()
                pending.pop(0)
                continue
            if self._used + fp > self.budget:
                st.close()
                break  # wait for memory to free up
            pending.pop(0)
            st.bind()
            st.thermalize(self.therm)
            self._used += fp
            self.peak_used = max(self.peak_used, self._used)
            res = results[req.id]
            res.admitted = clock() - t0
            res.footprint = fp
            active.append([req, st, fp, 0, None])


def poisson_stream(n_runs: int, seed: int, rate: float, L_range=(4, 20), h_range=(0.5, 4.0),
                   alphas=(1, 2, 4), samples=(1024, 2048, 4096, 8192, 16384),
                   n_steps: int = 50) -> List[Request]:
    """A seeded Poisson stream of run requests: exponential inter-arrival times
    with mean 1/rate seconds; per run L ~ U{L_range}, h ~ U[h_range], alpha and
    the number of samples drawn uniformly from the given choices, and its own
    parameter and chain seeds."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k in range(n_runs):
        t += rng.exponential(1.0 / rate)
        L = int(rng.integers(L_range[0], L_range[1] + 1))
        n_s = int(rng.choice(samples))
        h = float(rng.uniform(*h_range))
        alpha = int(rng.choice(alphas))
        out.append(Request(k, t, L, h, alpha, n_s, n_steps, int(rng.integers(1, 2**31)),
                           int(rng.integers(1, 2**31))))
    return out


requests_from_stream = poisson_stream
