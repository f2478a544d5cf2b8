"""Complex-parameter RBM with a holomorphic mapping theta -> psi: the oracle of
the complex holomorphic path (FP64 / complex128).

TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline timing).  Nothing
here is imported by the product library.

What it follows (paper sections and equations):
  * model: the RBM log-amplitude with complex a, b, W (complex parameters;
    holomorphic architectures, section on model parameters);
  * log-derivatives O_k = d ln psi / d theta_k (log-derivative equation), which
    for a holomorphic mapping satisfy the Cauchy-Riemann relations
    d ln psi / d Re theta = O, d ln psi / d Im theta = i O;
  * force f~_k = E[O_k^* (E - E[E])] (force-vector equation) and the gradient
    f = f~ for complex holomorphic parameters (complex co-gradient equation);
  * QGT G_ij = E[O_i^* (O_j - E[O_j])] (QGT estimator), = dJ^H dJ / N_s with the
    centred Jacobian (appendix QGTJacobian);
  * SR: G delta = f (complex holomorphic SR equation), theta <- theta - eta delta;
  * TDVP: G theta_dot = gamma f (TDVP equation of motion), gamma = -i for real
    time, -1 for imaginary time; Euler and Heun (second-order) Runge-Kutta
    steps (Runge-Kutta step equation).

Parameter vectors are complex128 in the packed layout [a | b | W (M x N)]
(both biases present).  Normalisation 1/N_s everywhere, as for the real path.
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import Optional

import numpy as np

from . import core, exact


def _lib():
    L = core.lib()
    if not getattr(L, "_holo_declared", False):
        P = ctypes.c_void_p
        i32, i64, u64, d = ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
        L.ora_log_psi_c.argtypes = [i32, i32, P, P, i64, P]
        L.ora_sample_c.argtypes = [i32, i32, P, i32, i32, P, i32, i32, i32, u64, u64, i32,
                                   i32, P, P, P, P, P]
        L.ora_local_energy_c.argtypes = [i32, i32, P, i32, i32, P, d, d, P, P, i64, P]
        L.ora_jacobian_c.argtypes = [i32, i32, P, P, i64, P]
        L._holo_declared = True
    return L


_ptr = core._ptr


@dataclasses.dataclass
class RbmC:
    """RBM with complex parameters, N visible and M hidden units."""
    N: int
    M: int
    params: np.ndarray  # complex128 [N + M + M N]

    def __post_init__(self):
        self.params = np.ascontiguousarray(self.params, dtype=np.complex128)
        if self.params.size != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters, got {self.params.size}")

    @property
    def n_params(self) -> int:
        return self.N + self.M + self.M * self.N

    def with_params(self, p) -> "RbmC":
        return RbmC(self.N, self.M, p)


def _cfg(rbm: RbmC, s) -> np.ndarray:
    return np.ascontiguousarray(s, dtype=np.int8).reshape(-1, rbm.N)


def log_psi(rbm: RbmC, s) -> np.ndarray:
    s = _cfg(rbm, s)
    out = np.zeros(s.shape[0], dtype=np.complex128)
    _lib().ora_log_psi_c(rbm.N, rbm.M, _ptr(rbm.params), _ptr(s), s.shape[0], _ptr(out))
    return out


def sample(rbm: RbmC, chains, S: int, K: int, seed: int, prop_base: int,
           rule: str = "local", bonds=None, chain_offset: int = 0,
           mode: str = "definition", log_accepts: bool = False) -> core.SampleResult:
    """Metropolis sampling of |psi|^2 (same draws as the real path)."""
    chains = np.array(chains, dtype=np.int8, copy=True, order="C")
    C, N = chains.shape
    r = 0 if rule == "local" else 1
    if r == 1 and bonds is None:
        raise ValueError("exchange rule needs bonds")
    b = np.ascontiguousarray(bonds if bonds is not None else np.zeros((1, 2)), dtype=np.int32)
    samples = np.zeros((C, S, N), dtype=np.int8)
    acc = np.zeros((C, S * K), dtype=np.uint8) if log_accepts else None
    margins = np.zeros(C)
    n_acc = np.zeros(C, dtype=np.int64)
    _lib().ora_sample_c(N, rbm.M, _ptr(rbm.params), r, b.shape[0], _ptr(b), C, S, K,
                        ctypes.c_uint64(seed), ctypes.c_uint64(prop_base), chain_offset,
                        0 if mode == "definition" else 1, _ptr(chains), _ptr(samples),
                        _ptr(acc), _ptr(margins), _ptr(n_acc))
    return core.SampleResult(chains, samples, acc, margins, n_acc)


def local_energy(rbm: RbmC, ham: core.Hamiltonian, s) -> np.ndarray:
    s = _cfg(rbm, s)
    out = np.zeros(s.shape[0], dtype=np.complex128)
    _lib().ora_local_energy_c(rbm.N, rbm.M, _ptr(rbm.params), ham.kind, ham.bonds.shape[0],
                              _ptr(ham.bonds), ham.J, ham.h, _ptr(ham.sublattice), _ptr(s),
                              s.shape[0], _ptr(out))
    return out


def jacobian(rbm: RbmC, s) -> np.ndarray:
    """O[k, p] = d ln psi(s_k) / d theta_p (complex)."""
    s = _cfg(rbm, s)
    O = np.zeros((s.shape[0], rbm.n_params), dtype=np.complex128)
    _lib().ora_jacobian_c(rbm.N, rbm.M, _ptr(rbm.params), _ptr(s), s.shape[0], _ptr(O))
    return O


# --------------------------------------------------------------------------
# Estimators
# --------------------------------------------------------------------------
def energy_stats(E: np.ndarray) -> dict:
    """Mean (complex; its real part is the energy), variance of E and error."""
    n = E.size
    mean = E.sum() / n
    var = float((np.abs(E - mean) ** 2).sum() / n)
    return dict(mean=mean, variance=var, error=np.sqrt(var / n))


def force(O: np.ndarray, E: np.ndarray) -> np.ndarray:
    """f = f~ = Cov[O, E] = (1/N_s) O^H (E - mean E) (holomorphic co-gradient)."""
    n = E.size
    dE = E - E.sum() / n
    return O.conj().T @ dE / n


def qgt_dense(O: np.ndarray) -> np.ndarray:
    """G = (1/N_s) dO^H dO, dO the column-centred Jacobian."""
    n = O.shape[0]
    dO = O - O.sum(axis=0) / n
    return dO.conj().T @ dO / n


def cg(matvec, f: np.ndarray, tol: float, maxiter: int):
    """Conjugate gradients for a Hermitian positive-definite operator, complex
    inner products <x, y> = x^H y; x0 = 0; stop at ||r|| <= tol ||f||."""
    x = np.zeros_like(f)
    r = f.copy()
    p = r.copy()
    rr = float(np.vdot(r, r).real)
    fn = np.sqrt(rr)
    it = 0
    if fn == 0.0:
        return x, 0, 0.0, True
    while np.sqrt(rr) > tol * fn and it < maxiter:
        Ap = matvec(p)
        alpha = rr / float(np.vdot(p, Ap).real)
        x = x + alpha * p
        r = r - alpha * Ap
        rr_new = float(np.vdot(r, r).real)
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    res = np.sqrt(rr) / fn
    return x, it, res, bool(res <= tol)


def solve_dense(O: np.ndarray, rhs: np.ndarray, diag_shift: float, tol: float,
                maxiter: Optional[int] = None):
    """(G + eps I) x = rhs by CG on the dense G (QGTJacobianDense, holomorphic)."""
    G = qgt_dense(O) + diag_shift * np.eye(O.shape[1])
    if maxiter is None:
        maxiter = min(rhs.size, 10000)
    return cg(lambda v: G @ v, rhs, tol, maxiter)


def cholesky_solve(O: np.ndarray, rhs: np.ndarray, diag_shift: float) -> np.ndarray:
    import scipy.linalg as sla
    A = qgt_dense(O) + diag_shift * np.eye(O.shape[1])
    return sla.cho_solve(sla.cho_factor(A, lower=True), rhs)


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


def vmc_step(rbm: RbmC, ham: core.Hamiltonian, chains, S: int, K: int, seed: int,
             prop_base: int, diag_shift: float, lr: float, tol: float,
             maxiter: Optional[int] = None, rule: str = "local", mode: str = "cached"):
    """sample -> local energies -> force -> G delta = f (dense QGT, CG) -> update."""
    res = sample(rbm, chains, S, K, seed, prop_base, rule, ham.bonds, mode=mode)
    flat = res.samples.reshape(-1, rbm.N)
    E = local_energy(rbm, ham, flat)
    O = jacobian(rbm, flat)
    f = force(O, E)
    delta, it, resid, _ = solve_dense(O, f, diag_shift, tol, maxiter)
    new = rbm.with_params(rbm.params - lr * delta)
    acc = res.n_accepted.sum() / (res.chains.shape[0] * S * K)
    return new, res.chains, StepReport(energy_stats(E), f, delta, it, resid, acc,
                                       res.samples, E)


def tdvp_rhs(rbm: RbmC, ham: core.Hamiltonian, chains, S: int, K: int, seed: int,
             prop_base: int, gamma: complex, diag_shift: float, tol: float,
             maxiter: Optional[int] = None, rule: str = "local", mode: str = "cached"):
    """theta_dot = F(theta): sample, then solve (G + eps I) x = f and return gamma x.
    Returns (theta_dot, new chains, StepReport with delta = x)."""
    res = sample(rbm, chains, S, K, seed, prop_base, rule, ham.bonds, mode=mode)
    flat = res.samples.reshape(-1, rbm.N)
    E = local_energy(rbm, ham, flat)
    O = jacobian(rbm, flat)
    f = force(O, E)
    x, it, resid, _ = solve_dense(O, f, diag_shift, tol, maxiter)
    acc = res.n_accepted.sum() / (res.chains.shape[0] * S * K)
    return gamma * x, res.chains, StepReport(energy_stats(E), f, x, it, resid, acc,
                                             res.samples, E)


def tdvp_step(rbm: RbmC, ham: core.Hamiltonian, chains, S: int, K: int, seed: int,
              prop_base: int, dt: float, gamma: complex, scheme: str, diag_shift: float,
              tol: float, maxiter: Optional[int] = None, rule: str = "local",
              mode: str = "cached"):
    """One Runge-Kutta step of the TDVP equation of motion.  Euler:
    theta += dt k1.  Heun: k1 = F(theta), k2 = F(theta + dt k1),
    theta += dt (k1 + k2) / 2.  Every evaluation of F draws S samples per chain
    (proposal counters advance by S K per evaluation).  Returns (new RbmC, new
    chains, list of StepReports, proposals used)."""
    k1, ch, r1 = tdvp_rhs(rbm, ham, chains, S, K, seed, prop_base, gamma, diag_shift, tol,
                          maxiter, rule, mode)
    if scheme == "euler":
        return rbm.with_params(rbm.params + dt * k1), ch, [r1], S * K
    if scheme != "heun":
        raise ValueError(scheme)
    mid = rbm.with_params(rbm.params + dt * k1)
    k2, ch, r2 = tdvp_rhs(mid, ham, ch, S, K, seed, prop_base + S * K, gamma, diag_shift, tol,
                          maxiter, rule, mode)
    return rbm.with_params(rbm.params + 0.5 * dt * (k1 + k2)), ch, [r1, r2], 2 * S * K


# --------------------------------------------------------------------------
# Exact references (full enumeration; the paper's ExactState)
# --------------------------------------------------------------------------
class ExactStateC:
    """Full-sum expectations over |psi(s)|^2 / Z for the complex RBM."""

    def __init__(self, rbm: RbmC, ham: core.Hamiltonian):
        self.rbm, self.ham = rbm, ham
        cfg = exact.all_configs(rbm.N)
        lp = log_psi(rbm, cfg)
        lp = lp - lp.real.max()
        self.psi = np.exp(lp)                   # unnormalised amplitudes
        w = np.abs(self.psi) ** 2
        self.p = w / w.sum()
        self.configs = cfg
        self.H = exact.hamiltonian_matrix(ham)

    def energy(self) -> float:
        v = self.psi
        return float((np.vdot(v, self.H @ v) / np.vdot(v, v)).real)

    def local_energies(self) -> np.ndarray:
        return (self.H @ self.psi) / self.psi

    def jacobian(self) -> np.ndarray:
        return jacobian(self.rbm, self.configs)

    def force(self) -> np.ndarray:
        O, E, p = self.jacobian(), self.local_energies(), self.p
        return (O - p @ O).conj().T @ (p * (E - p @ E))

    def qgt(self) -> np.ndarray:
        O, p = self.jacobian(), self.p
        dO = O - p @ O
        return dO.conj().T @ (p[:, None] * dO)


def exact_tdvp_step(rbm: RbmC, ham: core.Hamiltonian, dt: float, gamma: complex,
                    scheme: str, diag_shift: float = 0.0) -> RbmC:
    """One Euler / Heun step of the TDVP with exact expectations (no sampling),
    the dense solve done by numpy."""
    def F(r):
        ex = ExactStateC(r, ham)
        G = ex.qgt() + diag_shift * np.eye(r.n_params)
        return gamma * np.linalg.solve(G, ex.force())
    k1 = F(rbm)
    if scheme == "euler":
        return rbm.with_params(rbm.params + dt * k1)
    k2 = F(rbm.with_params(rbm.params + dt * k1))
    return rbm.with_params(rbm.params + 0.5 * dt * (k1 + k2))
