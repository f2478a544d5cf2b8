"""Python face of libnqs: one ``VMCState`` per C context.

PyTorch supplies device memory (the workspace and every input/output tensor)
and the HIP stream; the method itself runs in libnqs's kernels.  There is no
fallback: without a GPU or without ``libnqs.so`` every call raises.
"""
from __future__ import annotations

import ctypes
import dataclasses
import json
import time
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import (NqsError, NqsSrInfo, NqsStats, NqsStepCfg, NqsStepReport, NqsTdvpCfg,
                   NqsTdvpReport)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


@dataclasses.dataclass
class SrInfo:
    iterations: int
    converged: bool
    rel_residual: float


@dataclasses.dataclass
class StepReport:
    energy: dict
    sr: SrInfo
    status: int


def _stats_dict(s: NqsStats) -> dict:
    return dict(mean=s.mean, variance=s.variance, error=s.error, acceptance=s.acceptance)


class VMCState:
    """An RBM variational state with a Metropolis sampler on one GPU: real
    parameters (precision fp64, fp32 or bf16) or complex parameters with a
    holomorphic mapping (precision c128: parameters, gradients, directions,
    local energies, ln psi and Jacobians are complex128)."""

    def __init__(self, *, model: str, n_sites: int, bonds, J: float, h: float = 0.0,
                 sublattice=None, n_hidden: int, visible_bias: bool = True,
                 hidden_bias: bool = True, precision: str = "fp64", rule: str = "local",
                 n_chains: int, samples_per_chain: int, sweep_size: int, seed: int,
                 total_sz_zero: bool = False, qgt: str = "onthefly", device: int = 0,
                 stream: Optional[torch.cuda.Stream] = None, params=None, allocate: bool = True,
                 symmetries=None, alpha: Optional[int] = None, dense_solver: str = "cg"):
        """symmetries (int [G][n_sites] site permutations, row 0 the identity) with
        alpha: the symmetric RBM (alpha features over the group; n_hidden is then
        alpha * G, the plain RBM it runs as); its Jacobian is FP64 over the
        symmetric parameters and its QGT the dense one.  dense_solver ("cg" or
        "cholesky"): how dense QGT systems are solved."""
        if not torch.cuda.is_available():
            raise RuntimeError("libnqs needs a HIP device; none is visible")
        self.lib = _lib.load()
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.precision = precision
        self.n_sites, self.n_hidden = n_sites, n_hidden
        self.n_chains, self.samples_per_chain, self.sweep_size = n_chains, samples_per_chain, sweep_size
        self.complex = precision == "c128"
        self.symmetric = symmetries is not None
        self.rdtype = (torch.complex128 if self.complex else
                       torch.float64 if precision == "fp64" else torch.float32)
        self.jdtype = torch.float64 if self.symmetric else self.rdtype  # Jacobian entries
        if self.complex or self.symmetric:
            qgt = "jacobian_dense"
        if self.symmetric:
            self._perms = np.ascontiguousarray(symmetries, dtype=np.int32)
            if alpha is None:
                raise ValueError("a symmetric RBM needs alpha")
            n_hidden = alpha * self._perms.shape[0]
        self.alpha = alpha
        h_ctx = ctypes.c_void_p()
        st = self.lib.nqs_create(ctypes.byref(h_ctx), device, ctypes.c_void_p(self.stream.cuda_stream))
        if st:
            raise NqsError(st, "nqs_create failed")
        self.ctx = h_ctx
        b = np.ascontiguousarray(bonds, dtype=np.int32)
        self._bonds = b
        if model == "tfim":
            self._check(self.lib.nqs_set_tfim(self.ctx, n_sites, b.shape[0],
                                              b.ctypes.data_as(ctypes.c_void_p), J, h))
        elif model == "heisenberg":
            sub = None if sublattice is None else np.ascontiguousarray(sublattice, dtype=np.int8)
            self._check(self.lib.nqs_set_heisenberg(
                self.ctx, n_sites, b.shape[0], b.ctypes.data_as(ctypes.c_void_p), J,
                None if sub is None else sub.ctypes.data_as(ctypes.c_void_p)))
        else:
            raise ValueError(f"unknown model {model!r}")
        if self.symmetric:
            if self._perms.ndim != 2 or self._perms.shape[1] != n_sites:
                raise ValueError("symmetries must be [G][n_sites]")
            self._check(self.lib.nqs_set_rbm_symm(
                self.ctx, self._perms.shape[0], self._perms.ctypes.data_as(ctypes.c_void_p), alpha,
                int(visible_bias), int(hidden_bias), _lib.PRECISIONS[precision]))
        else:
            self._check(self.lib.nqs_set_rbm(self.ctx, n_hidden, int(visible_bias),
                                             int(hidden_bias), _lib.PRECISIONS[precision]))
        self._check(self.lib.nqs_set_sampler(self.ctx, _lib.RULES[rule], n_chains,
                                             samples_per_chain, sweep_size, seed,
                                             int(total_sz_zero)))
        self._check(self.lib.nqs_set_qgt(self.ctx, _lib.QGTS[qgt]))
        self._check(self.lib.nqs_set_dense_solver(self.ctx, _lib.DENSE_SOLVERS[dense_solver]))
        self.n_params = int(self.lib.nqs_num_params(self.ctx))
        self.workspace_bytes = int(self.lib.nqs_workspace_bytes(self.ctx))
        self.workspace = None
        self._pending_params = params
        if allocate:
            self.bind()

    def bind(self):
        """Allocate the workspace (the context's whole HBM footprint) and bind it."""
        if self.workspace is not None:
            return
        with torch.cuda.stream(self.stream):
            self.workspace = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8,
                                         device=self.device)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        self._check(self.lib.nqs_bind_workspace(self.ctx, ctypes.c_void_p(base + off),
                                                self.workspace_bytes))
        if self._pending_params is not None:
            self.set_params(self._pending_params)
            self._pending_params = None

    @classmethod
    def from_workload(cls, w, precision: Optional[str] = None, qgt: str = "onthefly",
                      device: int = 0, stream=None, params=None, n_chains: Optional[int] = None,
                      allocate: bool = True):
        """Build the state described by ``w`` (initial parameters included): any
        object with the attributes of ``lattice.RunSpec`` (model, n_sites,
        bonds(), J, h, sublattice(), n_hidden, precision, rule, n_chains,
        samples_per_chain, sweep_size, chain_seed, total_sz_zero, params())."""
        return cls(model=w.model, n_sites=w.n_sites, bonds=w.bonds(), J=w.J, h=w.h,
                   sublattice=w.sublattice(), n_hidden=w.n_hidden,
                   precision=precision or w.precision, rule=w.rule,
                   n_chains=n_chains or w.n_chains, samples_per_chain=w.samples_per_chain,
                   sweep_size=w.sweep_size, seed=w.chain_seed, total_sz_zero=w.total_sz_zero,
                   qgt=qgt, device=device, stream=stream,
                   params=w.params() if params is None else params, allocate=allocate)

    # ------------------------------------------------------------------
    def _check(self, st: int):
        if st != _lib.NQS_OK:
            msg = self.lib.nqs_last_error(self.ctx).decode()
            raise NqsError(st, msg)

    def close(self):
        """Destroy the context and release its workspace."""
        log = getattr(self, "_step_log", None)
        if log is not None:
            log["fh"].close()
            self._step_log = None
        if getattr(self, "ctx", None):
            self.lib.nqs_destroy(self.ctx)
            self.ctx = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def n_samples(self) -> int:
        return self.n_chains * self.samples_per_chain

    def _dev(self, t: torch.Tensor, dtype) -> torch.Tensor:
        return t.to(device=self.device, dtype=dtype).contiguous()

    # ------------------------------------------------------------------
    def set_params(self, p):
        if self.complex:  # complex128 values, passed as (real, imaginary) pairs
            if torch.is_tensor(p):
                p = torch.view_as_real(self._dev(p, torch.complex128)).contiguous()
                self._check(self.lib.nqs_set_params(self.ctx, _ptr(p), 1))
                return
            p = np.ascontiguousarray(np.asarray(p, dtype=np.complex128))
            if p.size != self.n_params:
                raise ValueError(f"expected {self.n_params} parameters")
            self._check(self.lib.nqs_set_params(self.ctx, p.ctypes.data_as(ctypes.c_void_p), 0))
            return
        p = np.ascontiguousarray(np.asarray(p, dtype=np.float64)) if not torch.is_tensor(p) else p
        if torch.is_tensor(p):
            p = self._dev(p, torch.float64)
            self._check(self.lib.nqs_set_params(self.ctx, _ptr(p), 1))
        else:
            if p.size != self.n_params:
                raise ValueError(f"expected {self.n_params} parameters")
            self._check(self.lib.nqs_set_params(self.ctx, p.ctypes.data_as(ctypes.c_void_p), 0))

    def get_params(self) -> np.ndarray:
        out = np.zeros(self.n_params, dtype=np.complex128 if self.complex else np.float64)
        self._check(self.lib.nqs_get_params(self.ctx, out.ctypes.data_as(ctypes.c_void_p), 0))
        return out

    def get_chains(self) -> np.ndarray:
        out = np.zeros((self.n_chains, self.n_sites), dtype=np.int8)
        self._check(self.lib.nqs_get_chains(self.ctx, out.ctypes.data_as(ctypes.c_void_p), 0))
        return out

    def set_chains(self, s):
        s = np.ascontiguousarray(s, dtype=np.int8)
        self._check(self.lib.nqs_set_chains(self.ctx, s.ctypes.data_as(ctypes.c_void_p), 0))

    def reset_chains(self):
        self._check(self.lib.nqs_reset_chains(self.ctx))

    @property
    def proposal_count(self) -> int:
        return int(self.lib.nqs_proposal_count(self.ctx))

    def get_state(self) -> bytes:
        n = ctypes.c_size_t(0)
        self._check(self.lib.nqs_get_state(self.ctx, None, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        self._check(self.lib.nqs_get_state(self.ctx, buf, ctypes.byref(n)))
        return buf.raw[: n.value]

    def set_state(self, blob: bytes):
        self._check(self.lib.nqs_set_state(self.ctx, blob, len(blob)))

    # ------------------------------------------------------------------
    def sample(self, n_discard: int = 0, return_samples: bool = True, log_accepts: bool = False):
        """Advance the chains; returns (samples [C, S, N] int8, accept log, acceptance)."""
        smp = None
        if return_samples:
            smp = torch.empty((self.n_chains, self.samples_per_chain, self.n_sites),
                              dtype=torch.int8, device=self.device)
        acc = None
        if log_accepts:
            acc = torch.empty((self.n_chains, self.samples_per_chain * self.sweep_size),
                              dtype=torch.uint8, device=self.device)
        a = ctypes.c_double(0.0)
        self._check(self.lib.nqs_sample(self.ctx, n_discard, _ptr(smp), _ptr(acc), ctypes.byref(a)))
        return smp, acc, a.value

    def thermalize(self, n_segments: int):
        """Advance the chains by n_segments * sweep_size unrecorded proposals."""
        self._check(self.lib.nqs_thermalize(self.ctx, n_segments))

    def load_samples(self, s: torch.Tensor):
        s = self._dev(s.reshape(-1, self.n_sites), torch.int8)
        self._check(self.lib.nqs_load_samples(self.ctx, _ptr(s), s.shape[0]))
        self._held = s

    def local_energy(self, s: torch.Tensor) -> torch.Tensor:
        s = self._dev(s.reshape(-1, self.n_sites), torch.int8)
        out = torch.empty(s.shape[0], dtype=torch.complex128 if self.complex else torch.float64,
                          device=self.device)
        self._check(self.lib.nqs_local_energy(self.ctx, _ptr(s), s.shape[0], _ptr(out)))
        return out

    def local_energy_noalloc(self, s: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
        """Local energies into the caller's `out` (float64 [n] on the device) through
        the entry point that allocates nothing (its staging is the library's static
        scratch)."""
        s = self._dev(s.reshape(-1, self.n_sites), torch.int8)
        if (out.dtype != torch.float64 or out.device != s.device or not out.is_contiguous()
                or out.numel() < s.shape[0]):
            raise ValueError("out must be a float64 device tensor with a slot per sample")
        self._check(self.lib.nqs_local_energy_noalloc(self.ctx, _ptr(s), s.shape[0], _ptr(out)))
        return out

    def log_psi(self, s: torch.Tensor) -> torch.Tensor:
        s = self._dev(s.reshape(-1, self.n_sites), torch.int8)
        out = torch.empty(s.shape[0], dtype=self.rdtype, device=self.device)
        self._check(self.lib.nqs_log_psi(self.ctx, _ptr(s), s.shape[0], _ptr(out)))
        return out

    def log_psi_vjp(self, s: torch.Tensor, g: torch.Tensor) -> torch.Tensor:
        s = self._dev(s.reshape(-1, self.n_sites), torch.int8)
        g = self._dev(g.reshape(-1), self.rdtype)
        out = torch.empty(self.n_params, dtype=self.rdtype, device=self.device)
        self._check(self.lib.nqs_log_psi_vjp(self.ctx, _ptr(s), s.shape[0], _ptr(g), _ptr(out)))
        return out

    def jacobian(self, s: torch.Tensor, center: bool = False) -> torch.Tensor:
        s = self._dev(s.reshape(-1, self.n_sites), torch.int8)
        out = torch.empty((s.shape[0], self.n_params), dtype=self.jdtype, device=self.device)
        self._check(self.lib.nqs_jacobian(self.ctx, _ptr(s), s.shape[0], _ptr(out), int(center)))
        return out

    def expect_and_grad(self, want_grad: bool = True):
        st = NqsStats()
        gt = torch.complex128 if self.complex else torch.float64
        g = torch.empty(self.n_params, dtype=gt, device=self.device) if want_grad else None
        self._check(self.lib.nqs_expect_and_grad(self.ctx, ctypes.byref(st), _ptr(g)))
        return _stats_dict(st), g

    def sr_update(self, qgt: str = "onthefly", diag_shift: float = 0.01, lr: float = 0.01,
                  tol: float = 1e-6, maxiter: int = 0, want_delta: bool = True,
                  allow_notconv: bool = False):
        info = NqsSrInfo()
        if self.complex or self.symmetric:
            qgt = "jacobian_dense"
        dt = torch.complex128 if self.complex else torch.float64
        d = torch.empty(self.n_params, dtype=dt, device=self.device) if want_delta else None
        st = self.lib.nqs_sr_update(self.ctx, _lib.QGTS[qgt], diag_shift, lr, tol, maxiter, _ptr(d),
                                    ctypes.byref(info))
        if not (st == _lib.NQS_OK or (allow_notconv and st == _lib.NQS_ENOTCONV)):
            self._check(st)
        return d, SrInfo(info.iterations, bool(info.converged), info.rel_residual)

    def vmc_step(self, qgt: str = "onthefly", diag_shift: float = 0.01, lr: float = 0.01,
                 tol: float = 1e-6, maxiter: int = 0) -> StepReport:
        if self.complex or self.symmetric:
            qgt = "jacobian_dense"
        cfg = NqsStepCfg(_lib.QGTS[qgt], diag_shift, lr, tol, maxiter)
        rep = NqsStepReport()
        log = getattr(self, "_step_log", None)
        if log is not None and log["stages"]:
            self.profile_enable(None)
        t0 = time.perf_counter()
        st = self.lib.nqs_vmc_step(self.ctx, ctypes.byref(cfg), ctypes.byref(rep))
        wall = time.perf_counter() - t0
        if st not in (_lib.NQS_OK, _lib.NQS_ENOTCONV):
            self._check(st)
        out = StepReport(_stats_dict(rep.energy),
                         SrInfo(rep.sr.iterations, bool(rep.sr.converged), rep.sr.rel_residual),
                         rep.status)
        if log is not None:
            self._write_step_log(out, wall)
        return out

    def tdvp_step(self, dt: float, gamma: complex = -1j, scheme: str = "heun",
                  diag_shift: float = 0.0, tol: float = 1e-8, maxiter: int = 0):
        """One TDVP step (complex models): returns a list with, per evaluation of
        the equation of motion, its energy (complex mean, variance, error,
        acceptance) and solve (iterations, converged, residual)."""
        g = complex(gamma)
        cfg = NqsTdvpCfg(_lib.RK_SCHEMES[scheme], dt, g.real, g.imag, diag_shift, tol, maxiter)
        rep = NqsTdvpReport()
        st = self.lib.nqs_tdvp_step(self.ctx, ctypes.byref(cfg), ctypes.byref(rep))
        if st not in (_lib.NQS_OK, _lib.NQS_ENOTCONV):
            self._check(st)
        out = []
        for l in range(rep.stages):
            e = _stats_dict(rep.energy[l])
            e["mean"] = complex(e["mean"], rep.energy_im[l])
            s = rep.solve[l]
            out.append(dict(energy=e, solve=SrInfo(s.iterations, bool(s.converged),
                                                   s.rel_residual)))
        return out

    # ------------------------------------------------------------------
    def open_step_log(self, path: str, stage_times: bool = False) -> None:
        """Append one JSON line per ``vmc_step`` to ``path``: step number, energy
        mean / variance / error, acceptance, CG iterations, residual and status,
        wall time; with ``stage_times`` also every kernel class's event-timed
        milliseconds in that step (the profiler then launches CG kernels one by
        one instead of replaying graphs, so those steps run slower)."""
        self.close_step_log()
        self._step_log = dict(fh=open(path, "a"), stages=stage_times, step=0)

    def close_step_log(self) -> None:
        log = getattr(self, "_step_log", None)
        if log is not None:
            log["fh"].close()
            if log["stages"]:
                self.profile_enable([])
        self._step_log = None

    def _write_step_log(self, rep: StepReport, wall: float) -> None:
        log = self._step_log
        log["step"] += 1
        rec = dict(step=log["step"], energy=rep.energy["mean"], variance=rep.energy["variance"],
                   error=rep.energy["error"], acceptance=rep.energy["acceptance"],
                   cg_iters=rep.sr.iterations, cg_rel_residual=rep.sr.rel_residual,
                   converged=rep.sr.converged, status=rep.status, wall_ms=wall * 1e3,
                   n_samples=self.n_samples, precision=self.precision)
        if log["stages"]:
            rec["stage_ms"] = {k: v["ms"] for k, v in self.profile_read().items() if v["launches"]}
        log["fh"].write(json.dumps(rec) + "\n")
        log["fh"].flush()


def _profile_enable(self, classes=None):
    """Time kernel classes with HIP events (None = all)."""
    mask = 0
    for k, name in enumerate(_lib.PROF_CLASSES):
        if classes is None or name in classes:
            mask |= 1 << k
    self._check(self.lib.nqs_profile_enable(self.ctx, mask))


def _profile_read(self) -> dict:
    n = len(_lib.PROF_CLASSES)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int64 * n)()
    self._check(self.lib.nqs_profile_read(self.ctx, ms, cnt, n))
    return {name: dict(ms=ms[k], launches=cnt[k]) for k, name in enumerate(_lib.PROF_CLASSES)}


def _set_cg_graphs(self, enable: bool = True) -> None:
    """Replay full batches of on-the-fly CG iterations from captured HIP graphs
    (default) or launch every kernel on the stream."""
    self._check(self.lib.nqs_set_cg_graphs(self.ctx, 1 if enable else 0))


def _probe_rate(self, kind: str) -> float:
    """Measured rate of one instruction kind on this device (see nqs_probe_rate):
    flops/s for "fp32_fma", "fp64_fma", "fp64_mfma", "bf16_mfma"; exponentials/s
    for "fp32_exp"."""
    v = ctypes.c_double(0.0)
    self._check(self.lib.nqs_probe_rate(self.ctx, _lib.PROBES[kind], ctypes.byref(v)))
    return v.value


VMCState.probe_rate = _probe_rate
VMCState.profile_enable = _profile_enable
VMCState.profile_read = _profile_read
VMCState.set_cg_graphs = _set_cg_graphs


def _set_cg_grouping(self, enable: bool = True) -> None:
    """Let batch_step run this run's on-the-fly CG iterations in launches
    grouped with the other runs of the step (default; BF16 and FP32 forms) or
    make it run its own launches.  The results are identical either way."""
    self._check(self.lib.nqs_set_cg_grouping(self.ctx, 1 if enable else 0))


VMCState.set_cg_grouping = _set_cg_grouping


def _step_cfg(c: dict) -> NqsStepCfg:
    return NqsStepCfg(_lib.QGTS[c.get("qgt", "onthefly")], c.get("diag_shift", 0.01),
                      c.get("lr", 0.01), c.get("tol", 1e-6), c.get("maxiter", 0))


def _step_report(lib, st: VMCState, r) -> StepReport:
    if r.status not in (_lib.NQS_OK, _lib.NQS_ENOTCONV):
        raise NqsError(r.status, lib.nqs_last_error(st.ctx).decode())
    return StepReport(_stats_dict(r.energy),
                      SrInfo(r.sr.iterations, bool(r.sr.converged), r.sr.rel_residual), r.status)


def step_begin(state: VMCState, cfg: dict) -> None:
    """Issue one VMC step on the state's stream and return at once
    (``nqs_step_begin``); ``step_poll`` advances it and reports its end."""
    c = _step_cfg(cfg)
    state._check(state.lib.nqs_step_begin(state.ctx, ctypes.byref(c)))


def step_poll(states: Sequence[VMCState], wait: bool = True) -> dict:
    """Advance the steps in flight on ``states`` (``nqs_step_poll``); returns
    {index: StepReport} for the steps that have completed (with ``wait``, at
    least one unless none is in flight)."""
    n = len(states)
    if n == 0:
        return {}
    lib = states[0].lib
    ctxs = (ctypes.c_void_p * n)(*[s.ctx.value for s in states])
    reps = (NqsStepReport * n)()
    done = (ctypes.c_int32 * n)()
    st = lib.nqs_step_poll(ctxs, n, 1 if wait else 0, reps, done)
    if st == _lib.NQS_EINVAL and not any(done):
        raise NqsError(st, "nqs_step_poll: invalid arguments")
    return {k: _step_report(lib, states[k], reps[k]) for k in range(n) if done[k]}


def batch_step(states: Sequence[VMCState], cfgs: Sequence[dict]) -> list:
    """One SR step for every state, issued in lock-step across their streams."""
    n = len(states)
    if n == 0:
        return []
    lib = states[0].lib
    ctxs = (ctypes.c_void_p * n)(*[s.ctx.value for s in states])
    c_cfgs = (NqsStepCfg * n)()
    for k, c in enumerate(cfgs):
        c_cfgs[k] = NqsStepCfg(_lib.QGTS[c.get("qgt", "onthefly")], c.get("diag_shift", 0.01),
                               c.get("lr", 0.01), c.get("tol", 1e-6), c.get("maxiter", 0))
    reps = (NqsStepReport * n)()
    lib.nqs_batch_step(ctxs, n, c_cfgs, reps)
    out = []
    for k in range(n):
        r = reps[k]
        if r.status not in (_lib.NQS_OK, _lib.NQS_ENOTCONV):
            msg = lib.nqs_last_error(states[k].ctx).decode()
            raise NqsError(r.status, f"context {k}: {msg}")
        out.append(StepReport(_stats_dict(r.energy),
                              SrInfo(r.sr.iterations, bool(r.sr.converged), r.sr.rel_residual),
                              r.status))
    return out
