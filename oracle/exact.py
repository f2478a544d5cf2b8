"""Exact references for small systems: Hamiltonian matrices built from Pauli
Kronecker products, exact diagonalisation, full enumeration of the Born
distribution (the paper's ExactState), and the closed-form ground energy of
the periodic transverse-field Ising chain.

TEST INFRASTRUCTURE ONLY.

Basis convention: basis index n in [0, 2^N); site i is bit N-1-i of n (site 0
is the leftmost Kronecker factor); bit 0 <-> s_i = +1 (sigma^z eigenvalue +1).
"""
from __future__ import annotations

import itertools
from typing import Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import core

_I = sp.identity(2, format="csr", dtype=np.complex128)
_X = sp.csr_matrix(np.array([[0, 1], [1, 0]], dtype=np.complex128))
_Y = sp.csr_matrix(np.array([[0, -1j], [1j, 0]], dtype=np.complex128))
_Z = sp.csr_matrix(np.array([[1, 0], [0, -1]], dtype=np.complex128))


def site_op(op, i: int, N: int):
    """op acting on site i of N (identity elsewhere)."""
    left = sp.identity(2 ** i, format="csr", dtype=np.complex128)
    right = sp.identity(2 ** (N - 1 - i), format="csr", dtype=np.complex128)
    return sp.kron(sp.kron(left, op, format="csr"), right, format="csr")


def _real(H):
    H = H.tocsr()
    if H.nnz and np.abs(H.data.imag).max() > 1e-12:
        raise AssertionError("Hamiltonian is not real")
    return sp.csr_matrix((H.data.real, H.indices, H.indptr), shape=H.shape)


def tfim_matrix(N: int, bonds, J: float, h: float):
    """H = J sum_<ab> Z_a Z_b - h sum_i X_i (sparse, real)."""
    H = sp.csr_matrix((2 ** N, 2 ** N), dtype=np.complex128)
    for a, b in bonds:
        H = H + J * (site_op(_Z, int(a), N) @ site_op(_Z, int(b), N))
    for i in range(N):
        H = H - h * site_op(_X, i, N)
    return _real(H)


def heisenberg_matrix(N: int, bonds, J: float, sublattice: Optional[np.ndarray] = None):
    """H = J sum_<ab> (X X + Y Y + Z Z); with a sublattice array, the rotated
    operator U H U with U = prod over sublattice-1 sites of Z."""
    H = sp.csr_matrix((2 ** N, 2 ** N), dtype=np.complex128)
    for a, b in bonds:
        a, b = int(a), int(b)
        for P in (_X, _Y, _Z):
            H = H + J * (site_op(P, a, N) @ site_op(P, b, N))
    if sublattice is not None:
        U = sp.identity(2 ** N, format="csr", dtype=np.complex128)
        for i in range(N):
            if sublattice[i]:
                U = U @ site_op(_Z, i, N)
        H = U @ H @ U
    return _real(H)


def hamiltonian_matrix(ham: core.Hamiltonian):
    if ham.kind == 0:
        return tfim_matrix(ham.n_sites, ham.bonds, ham.J, ham.h)
    return heisenberg_matrix(ham.n_sites, ham.bonds, ham.J, ham.sublattice)


def all_configs(N: int) -> np.ndarray:
    """All 2^N configurations in basis order, int8 [2^N, N]."""
    n = np.arange(2 ** N)
    bits = (n[:, None] >> (N - 1 - np.arange(N))[None, :]) & 1
    return (1 - 2 * bits).astype(np.int8)


def sz0_mask(N: int) -> np.ndarray:
    return all_configs(N).astype(np.int64).sum(axis=1) == 0


def ground_energy(H, k: int = 1) -> np.ndarray:
    dim = H.shape[0]
    if dim <= 1024:
        w = np.linalg.eigvalsh(H.toarray())
        return w[:k]
    w = spla.eigsh(H, k=k, which="SA", return_eigenvectors=False, tol=1e-12)
    return np.sort(w)


def tfim_chain_ground_energy(N: int, J: float, h: float) -> float:
    """Closed form for the periodic TFIM chain with even N (Pfeuty 1970):
    E0 = -sum_{m=0}^{N-1} sqrt(J^2 + h^2 - 2 J h cos(pi (2m+1) / N))."""
    m = np.arange(N)
    return float(-np.sqrt(J * J + h * h - 2 * J * h * np.cos(np.pi * (2 * m + 1) / N)).sum())


class ExactState:
    """Full-sum expectations over the Born distribution |psi(s)|^2 / Z
    (the paper's ExactState), optionally restricted to total_sz = 0."""

    def __init__(self, rbm: core.Rbm, ham: core.Hamiltonian, sz0: bool = False):
        self.rbm, self.ham = rbm, ham
        N = rbm.N
        cfg = all_configs(N)
        self.mask = sz0_mask(N) if sz0 else np.ones(2 ** N, dtype=bool)
        lp = core.log_psi(rbm, cfg)
        lp = np.where(self.mask, lp, -np.inf)
        w = np.exp(2 * (lp - lp.max()))
        self.p = w / w.sum()
        self.psi = np.exp(lp - lp.max())
        self.configs = cfg
        self.H = hamiltonian_matrix(ham)

    def energy(self) -> float:
        """<psi|H|psi> / <psi|psi> with the Kronecker-product matrix."""
        v = self.psi
        return float(v @ (self.H @ v) / (v @ v))

    def local_energies(self) -> np.ndarray:
        """E(s) = (H psi)(s) / psi(s) for every s in the support."""
        v = self.psi
        Hv = self.H @ v
        out = np.full(v.size, np.nan)
        out[self.mask] = Hv[self.mask] / v[self.mask]
        return out

    def jacobian(self) -> np.ndarray:
        return core.jacobian(self.rbm, self.configs)

    def force(self) -> np.ndarray:
        """2 Cov_p[O, E] summed exactly over the support."""
        O = self.jacobian()[self.mask]
        E = self.local_energies()[self.mask]
        p = self.p[self.mask]
        Om = p @ O
        Em = p @ E
        return 2.0 * ((O - Om).T @ (p * (E - Em)))

    def qgt(self) -> np.ndarray:
        O = self.jacobian()[self.mask]
        p = self.p[self.mask]
        dO = O - p @ O
        return dO.T @ (p[:, None] * dO)

    def expectation_of(self, f_values: np.ndarray) -> float:
        return float(self.p[self.mask] @ f_values[self.mask])


def enumerate_configs(N: int, n_up: Optional[int] = None):
    """Iterator over configurations with an optional fixed number of up spins."""
    for bits in itertools.product((1, -1), repeat=N):
        if n_up is None or sum(b > 0 for b in bits) == n_up:
            yield np.array(bits, dtype=np.int8)
