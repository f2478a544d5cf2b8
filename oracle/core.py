"""Python face of the FP64 oracle: ctypes calls into ``liboracle.so`` for the
per-configuration work and plain numpy / scipy linear algebra for the
estimators and the stochastic-reconfiguration solve.

TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline timing).  Nothing
here is imported by the product library.

Parameter vectors handed to these functions use the packed layout
[a (if visible bias) | b (if hidden bias) | W (M x N row-major)];
``Rbm.full()`` expands to the full layout with zero biases where absent.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i32, i64, u64 = ctypes.c_int, ctypes.c_int64, ctypes.c_uint64
        L.ora_num_threads.restype = i32
        L.ora_philox4x32_10.argtypes = [P, u64, P]
        L.ora_init_chains.argtypes = [i32, i32, u64, i32, i32, P]
        L.ora_log_psi.argtypes = [i32, i32, P, P, i64, P]
        L.ora_sample.argtypes = [i32, i32, P, i32, i32, P, i32, i32, i32, u64, u64, i32,
                                 i32, P, P, P, P, P]
        L.ora_local_energy.argtypes = [i32, i32, P, i32, i32, P, ctypes.c_double,
                                       ctypes.c_double, P, P, i64, P]
        L.ora_jacobian.argtypes = [i32, i32, P, P, i64, P]
        _LIB = L
    return _LIB


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return lib().ora_num_threads()


# --------------------------------------------------------------------------
# Model and Hamiltonian descriptions
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Rbm:
    """Real RBM with N visible and M hidden units (packed parameters)."""
    N: int
    M: int
    params: np.ndarray
    visible_bias: bool = True
    hidden_bias: bool = True

    def __post_init__(self):
        self.params = np.ascontiguousarray(self.params, dtype=np.float64)
        if self.params.size != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters, got {self.params.size}")

    @property
    def n_params(self) -> int:
        return (self.N if self.visible_bias else 0) + (self.M if self.hidden_bias else 0) \
            + self.M * self.N

    def full(self) -> np.ndarray:
        """Full layout [a | b | W] with zeros for absent biases."""
        N, M = self.N, self.M
        out = np.zeros(N + M + M * N)
        k = 0
        if self.visible_bias:
            out[:N] = self.params[:N]
            k = N
        if self.hidden_bias:
            out[N:N + M] = self.params[k:k + M]
            k += M
        out[N + M:] = self.params[k:]
        return out

    def pack_columns(self) -> np.ndarray:
        """Indices of the packed parameters inside the full layout."""
        N, M = self.N, self.M
        idx = []
        if self.visible_bias:
            idx.append(np.arange(N))
        if self.hidden_bias:
            idx.append(N + np.arange(M))
        idx.append(N + M + np.arange(M * N))
        return np.concatenate(idx)

    def with_params(self, p: np.ndarray) -> "Rbm":
        return Rbm(self.N, self.M, p, self.visible_bias, self.hidden_bias)


@dataclasses.dataclass
class Hamiltonian:
    """TFIM (kind 0) or Heisenberg (kind 1, optional Marshall sublattice)."""
    kind: int
    n_sites: int
    bonds: np.ndarray
    J: float
    h: float = 0.0
    sublattice: Optional[np.ndarray] = None

    def __post_init__(self):
        self.bonds = np.ascontiguousarray(self.bonds, dtype=np.int32)
        if self.sublattice is not None:
            self.sublattice = np.ascontiguousarray(self.sublattice, dtype=np.int8)

    @staticmethod
    def tfim(n_sites, bonds, J, h):
        return Hamiltonian(0, n_sites, bonds, J, h)

    @staticmethod
    def heisenberg(n_sites, bonds, J, sublattice=None):
        return Hamiltonian(1, n_sites, bonds, J, 0.0, sublattice)


# --------------------------------------------------------------------------
# Thin wrappers over the C routines
# --------------------------------------------------------------------------
def philox(ctr, seed: int) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().ora_philox4x32_10(_ptr(c), ctypes.c_uint64(seed), _ptr(out))
    return out


def init_chains(N: int, C: int, seed: int, chain_offset: int = 0,
                total_sz_zero: bool = False) -> np.ndarray:
    out = np.zeros((C, N), dtype=np.int8)
    lib().ora_init_chains(N, C, seed, chain_offset, int(total_sz_zero), _ptr(out))
    return out


def log_psi(rbm: Rbm, s: np.ndarray) -> np.ndarray:
    s = np.ascontiguousarray(s, dtype=np.int8).reshape(-1, rbm.N)
    full = rbm.full()
    out = np.zeros(s.shape[0])
    lib().ora_log_psi(rbm.N, rbm.M, _ptr(full), _ptr(s), s.shape[0], _ptr(out))
    return out


@dataclasses.dataclass
class SampleResult:
    chains: np.ndarray        # [C, N] final configurations
    samples: np.ndarray       # [C, S, N]
    accepts: Optional[np.ndarray]  # [C, S*K] uint8
    margins: np.ndarray       # [C] smallest |u - ratio^2|
    n_accepted: np.ndarray    # [C]


def sample(rbm: Rbm, chains: np.ndarray, S: int, K: int, seed: int, prop_base: int,
           rule: str = "local", bonds: Optional[np.ndarray] = None, chain_offset: int = 0,
           mode: str = "definition", log_accepts: bool = False) -> SampleResult:
    """Metropolis sampling; ``chains`` is copied, not modified."""
    chains = np.array(chains, dtype=np.int8, copy=True, order="C")
    C, N = chains.shape
    if N != rbm.N:
        raise ValueError("chain width differs from the model")
    r = 0 if rule == "local" else 1
    if r == 1 and bonds is None:
        raise ValueError("exchange rule needs bonds")
    b = np.ascontiguousarray(bonds if bonds is not None else np.zeros((1, 2)), dtype=np.int32)
    samples = np.zeros((C, S, N), dtype=np.int8)
    acc = np.zeros((C, S * K), dtype=np.uint8) if log_accepts else None
    margins = np.zeros(C)
    n_acc = np.zeros(C, dtype=np.int64)
    full = rbm.full()
    lib().ora_sample(N, rbm.M, _ptr(full), r, b.shape[0], _ptr(b), C, S, K,
                     ctypes.c_uint64(seed), ctypes.c_uint64(prop_base), chain_offset,
                     0 if mode == "definition" else 1, _ptr(chains), _ptr(samples),
                     _ptr(acc), _ptr(margins), _ptr(n_acc))
    return SampleResult(chains, samples, acc, margins, n_acc)


def local_energy(rbm: Rbm, ham: Hamiltonian, s: np.ndarray) -> np.ndarray:
    s = np.ascontiguousarray(s, dtype=np.int8).reshape(-1, rbm.N)
    full = rbm.full()
    out = np.zeros(s.shape[0])
    lib().ora_local_energy(rbm.N, rbm.M, _ptr(full), ham.kind, ham.bonds.shape[0],
                           _ptr(ham.bonds), ham.J, ham.h, _ptr(ham.sublattice), _ptr(s),
                           s.shape[0], _ptr(out))
    return out


def jacobian(rbm: Rbm, s: np.ndarray) -> np.ndarray:
    """O[k, p] = d ln psi(s_k) / d p for the packed parameters."""
    s = np.ascontiguousarray(s, dtype=np.int8).reshape(-1, rbm.N)
    N, M = rbm.N, rbm.M
    full = rbm.full()
    O = np.zeros((s.shape[0], N + M + M * N))
    lib().ora_jacobian(N, M, _ptr(full), _ptr(s), s.shape[0], _ptr(O))
    if rbm.visible_bias and rbm.hidden_bias:
        return O
    return np.ascontiguousarray(O[:, rbm.pack_columns()])


# --------------------------------------------------------------------------
# Estimators (paper, "Estimating observables"; 1/N_s normalisation)
# --------------------------------------------------------------------------
def energy_stats(E: np.ndarray) -> dict:
    """Monte Carlo mean, variance and standard error of the mean."""
    E = np.asarray(E, dtype=np.float64)
    n = E.size
    mean = E.sum() / n
    var = ((E - mean) ** 2).sum() / n
    return dict(mean=mean, variance=var, error=np.sqrt(var / n))


def force(O: np.ndarray, E: np.ndarray) -> np.ndarray:
    """Energy gradient for real parameters: 2 Re Cov[O, E] = 2/N_s O^T (E - mean E)."""
    n = E.size
    dE = E - E.sum() / n
    return 2.0 * (O.T @ dE) / n


def qgt_dense(O: np.ndarray) -> np.ndarray:
    """S = (1/N_s) dO^T dO with dO the column-centred Jacobian (real part)."""
    n = O.shape[0]
    dO = O - O.sum(axis=0) / n
    return dO.T @ dO / n


def qgt_matvec(O: np.ndarray, v: np.ndarray, diag_shift: float = 0.0) -> np.ndarray:
    """On-the-fly product (appendix on QGTOnTheFly):
    w = J v / N_s;  dw = w - mean(w);  G v = J^T dw;  plus the diagonal shift."""
    n = O.shape[0]
    w = O @ v / n
    dw = w - w.sum() / n
    return O.T @ dw + diag_shift * v


def cg(matvec, f: np.ndarray, tol: float, maxiter: int, x0: Optional[np.ndarray] = None):
    """Conjugate gradients for a symmetric positive-definite operator.

    Starts at x0 (zero by default) and stops once ||r||_2 <= tol * ||f||_2 or
    after ``maxiter`` iterations.  Returns (x, iterations, ||r|| / ||f||,
    converged)."""
    x = np.zeros_like(f) if x0 is None else np.array(x0, dtype=np.float64)
    r = f - matvec(x) if x0 is not None else f.copy()
    p = r.copy()
    rr = r @ r
    fn = np.sqrt(f @ f)
    it = 0
    if fn == 0.0:
        return x, 0, 0.0, True
    while np.sqrt(rr) > tol * fn and it < maxiter:
        Ap = matvec(p)
        alpha = rr / (p @ Ap)
        x = x + alpha * p
        r = r - alpha * Ap
        rr_new = r @ r
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    res = np.sqrt(rr) / fn
    return x, it, res, bool(res <= tol)


def cholesky_solve(S: np.ndarray, f: np.ndarray, diag_shift: float) -> np.ndarray:
    import scipy.linalg as sla
    A = S + diag_shift * np.eye(S.shape[0])
    c = sla.cho_factor(A, lower=True)
    return sla.cho_solve(c, f)


def sr_direction(O: np.ndarray, E: np.ndarray, diag_shift: float, tol: float,
                 maxiter: Optional[int] = None):
    """Solve (Re S + eps I) delta = f with CG on the on-the-fly product."""
    f = force(O, E)
    if maxiter is None:
        maxiter = min(f.size, 10000)
    delta, it, res, conv = cg(lambda v: qgt_matvec(O, v, diag_shift), f, tol, maxiter)
    return f, delta, it, res, conv


# --------------------------------------------------------------------------
# One VMC step with SR (paper, ground-state search section)
# --------------------------------------------------------------------------
@dataclasses.dataclass
class StepReport:
    energy: dict
    force: np.ndarray
    delta: np.ndarray
    cg_iters: int
    cg_residual: float
    acceptance: float
    samples: np.ndarray
    eloc: np.ndarray


def vmc_step(rbm: Rbm, ham: Hamiltonian, chains: np.ndarray, S: int, K: int, seed: int,
             prop_base: int, rule: str, diag_shift: float, lr: float, tol: float,
             maxiter: Optional[int] = None, mode: str = "cached"):
    """sample -> local energies -> statistics -> force -> SR solve -> update.

    Returns (new Rbm, new chains, StepReport)."""
    res = sample(rbm, chains, S, K, seed, prop_base, rule, ham.bonds, mode=mode)
    flat = res.samples.reshape(-1, rbm.N)
    E = local_energy(rbm, ham, flat)
    O = jacobian(rbm, flat)
    f, delta, it, resid, _ = sr_direction(O, E, diag_shift, tol, maxiter)
    new = rbm.with_params(rbm.params - lr * delta)
    acc = res.n_accepted.sum() / (chains.shape[0] * S * K)
    rep = StepReport(energy_stats(E), f, delta, it, resid, acc, res.samples, E)
    return new, res.chains, rep
