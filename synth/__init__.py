"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module holds no arithmetic of the method (no amplitudes, energies,
gradients or solves).  It only builds problem definitions and random inputs:
lattice bond lists, sublattice labels, initial RBM parameters and batches of
spin configurations, plus the named workloads used by tests and the benchmark.

Conventions (NetKet 3 paper, section "Quantum-mechanical primitives"):
  * spin-1/2 configurations are int8 vectors with entries in {+1, -1};
  * RBM parameters are one flat float64 vector laid out as
    [a (N, if visible bias) | b (M, if hidden bias) | W (M x N, row-major)],
    the contiguous ("dense") layout the paper describes for its Jacobian-based
    QGT;
  * periodic lattices: the 1D chain has bonds (i, i+1 mod N); the L x L square
    lattice has bonds (x,y)-(x+1,y) and (x,y)-(x,y+1), each listed once
    (requires L >= 3 so no bond is listed twice).
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

__all__ = [
    "chain_bonds", "square_bonds", "chain_sublattice", "square_sublattice",
    "n_params", "rbm_params", "rbm_params_c", "random_configs", "chain_translations",
    "square_translations", "symm_params", "sz0_configs", "Workload",
    "WORKLOADS",
]


def chain_bonds(n: int) -> np.ndarray:
    """Periodic chain of ``n`` sites: bonds (i, i+1 mod n), int32 [n, 2]."""
    if n < 3:
        raise ValueError("a periodic chain needs at least 3 sites")
    i = np.arange(n, dtype=np.int32)
    return np.stack([i, (i + 1) % n], axis=1).astype(np.int32)


def square_bonds(L: int) -> np.ndarray:
    """Periodic L x L square lattice, site = x + L*y; int32 [2*L*L, 2]."""
    if L < 3:
        raise ValueError("a periodic square lattice needs L >= 3")
    bonds = []
    for y in range(L):
        for x in range(L):
            s = x + L * y
            bonds.append((s, (x + 1) % L + L * y))
            bonds.append((s, x + L * ((y + 1) % L)))
    return np.asarray(bonds, dtype=np.int32)


def chain_sublattice(n: int) -> np.ndarray:
    """Sublattice label i mod 2 (bipartite for even n); int8 [n]."""
    return (np.arange(n) % 2).astype(np.int8)


def square_sublattice(L: int) -> np.ndarray:
    """Sublattice label (x + y) mod 2; int8 [L*L]."""
    x = np.arange(L * L) % L
    y = np.arange(L * L) // L
    return ((x + y) % 2).astype(np.int8)


def chain_translations(n: int) -> np.ndarray:
    """Translations of the periodic chain as site permutations: row g maps site k
    to k + g mod n (row 0 the identity); int32 [n, n]."""
    k = np.arange(n)
    return np.stack([(k + g) % n for g in range(n)]).astype(np.int32)


def square_translations(L: int) -> np.ndarray:
    """Translations of the periodic L x L square lattice (site = x + L*y): row
    g = dx + L*dy maps (x, y) to (x+dx, y+dy) mod L; int32 [L*L, L*L]."""
    x = np.arange(L * L) % L
    y = np.arange(L * L) // L
    rows = [((x + dx) % L) + L * ((y + dy) % L) for dy in range(L) for dx in range(L)]
    return np.stack(rows).astype(np.int32)


def symm_params(n_sites: int, alpha: int, seed: int, sigma: float = 0.01,
                visible_bias: bool = True, hidden_bias: bool = True) -> np.ndarray:
    """Initial parameters of a symmetric RBM, packed [a (1) | b (alpha) | W
    (alpha x n_sites)], drawn i.i.d. normal(0, sigma)."""
    P = (1 if visible_bias else 0) + (alpha if hidden_bias else 0) + alpha * n_sites
    return np.random.default_rng(seed).normal(0.0, sigma, size=P).astype(np.float64)


def n_params(n_sites: int, n_hidden: int, visible_bias: bool = True,
             hidden_bias: bool = True) -> int:
    return (n_sites if visible_bias else 0) + (n_hidden if hidden_bias else 0) \
        + n_hidden * n_sites


def rbm_params(n_sites: int, n_hidden: int, seed: int, sigma: float = 0.01,
               visible_bias: bool = True, hidden_bias: bool = True) -> np.ndarray:
    """Initial parameters drawn i.i.d. normal(0, sigma) (sigma = std dev)."""
    rng = np.random.default_rng(seed)
    P = n_params(n_sites, n_hidden, visible_bias, hidden_bias)
    return rng.normal(0.0, sigma, size=P).astype(np.float64)


def rbm_params_c(n_sites: int, n_hidden: int, seed: int, sigma: float = 0.01) -> np.ndarray:
    """Complex initial parameters (both biases): real and imaginary parts drawn
    i.i.d. normal(0, sigma), as one [P, 2] array of (real, imaginary) pairs."""
    rng = np.random.default_rng(seed)
    P = n_params(n_sites, n_hidden)
    z = rng.normal(0.0, sigma, size=(P, 2))
    return (z[:, 0] + 1j * z[:, 1]).astype(np.complex128)


def random_configs(n: int, n_sites: int, seed: int) -> np.ndarray:
    """Uniform random spin configurations, int8 [n, n_sites] in {+1,-1}."""
    rng = np.random.default_rng(seed)
    return (1 - 2 * rng.integers(0, 2, size=(n, n_sites))).astype(np.int8)


def sz0_configs(n: int, n_sites: int, seed: int) -> np.ndarray:
    """Random zero-magnetisation configurations (n_sites even)."""
    if n_sites % 2:
        raise ValueError("total_sz = 0 needs an even number of sites")
    rng = np.random.default_rng(seed)
    base = np.array([1] * (n_sites // 2) + [-1] * (n_sites // 2), dtype=np.int8)
    out = np.empty((n, n_sites), dtype=np.int8)
    for k in range(n):
        out[k] = rng.permutation(base)
    return out


@dataclasses.dataclass(frozen=True)
class Workload:
    """One named synthetic workload (all sizes explicit)."""
    name: str
    model: str             # "tfim" or "heisenberg"
    lattice: str           # "chain" or "square"
    L: int                 # chain length or square side
    J: float
    h: float               # transverse field (TFIM only)
    alpha: int             # hidden-unit density M = alpha * N
    n_chains: int
    samples_per_chain: int
    sweep_size: int        # proposals between recorded samples
    rule: str              # "local" or "exchange"
    precision: str         # "fp64", "fp32", "bf16" or "c128" (complex parameters)
    param_seed: int = 1
    chain_seed: int = 2
    sigma: float = 0.01
    diag_shift: float = 0.01
    lr: float = 0.01
    cg_tol: float = 1e-6
    marshall: bool = False
    total_sz_zero: bool = False
    thermalize_segments: int = 100

    @property
    def n_sites(self) -> int:
        return self.L if self.lattice == "chain" else self.L * self.L

    @property
    def n_hidden(self) -> int:
        return self.alpha * self.n_sites

    @property
    def n_samples(self) -> int:
        return self.n_chains * self.samples_per_chain

    @property
    def n_params(self) -> int:
        return n_params(self.n_sites, self.n_hidden)

    def bonds(self) -> np.ndarray:
        return chain_bonds(self.L) if self.lattice == "chain" else square_bonds(self.L)

    def sublattice(self) -> Optional[np.ndarray]:
        if not self.marshall:
            return None
        return chain_sublattice(self.L) if self.lattice == "chain" else square_sublattice(self.L)

    def params(self) -> np.ndarray:
        if self.precision == "c128":
            return rbm_params_c(self.n_sites, self.n_hidden, self.param_seed, self.sigma)
        return rbm_params(self.n_sites, self.n_hidden, self.param_seed, self.sigma)

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


WORKLOADS = {
    # 1D TFIM periodic chain N=10, J=h=1, RBM alpha=1, 16 chains x 64 samples,
    # 10 proposals between samples, plain FP64.
    "tfim1d_n10": Workload("tfim1d_n10", "tfim", "chain", 10, 1.0, 1.0, 1, 16, 64,
                           10, "local", "fp64"),
    # 2D TFIM 10x10 periodic, J=1, h=3.044, RBM alpha=2 (200 hidden),
    # 4096 chains x 4 samples, N=100 proposals between samples.
    "tfim2d_l10": Workload("tfim2d_l10", "tfim", "square", 10, 1.0, 3.044, 2, 4096, 4,
                           100, "local", "fp64"),
    # 2D Heisenberg 16x16 periodic, Marshall rotated, exchange moves, alpha=4,
    # 16384 chains x 1 sample, 256 proposals between samples, BF16 form.
    "heis2d_l16": Workload("heis2d_l16", "heisenberg", "square", 16, 1.0, 0.0, 4, 16384, 1,
                           256, "exchange", "bf16", marshall=True, total_sz_zero=True),
    # 1D Heisenberg chain N=64 periodic, Marshall rotated, alpha=8 (512 hidden),
    # 16384 samples, FP32 (dense Jacobian / Gram form).
    "heis1d_n64": Workload("heis1d_n64", "heisenberg", "chain", 64, 1.0, 0.0, 8, 4096, 4,
                           64, "exchange", "fp32", marshall=True, total_sz_zero=True),
    # 1D TFIM chain L=64, J=h=1, complex RBM alpha=1 (holomorphic), 1024 chains x
    # 16 samples = 2^14, L proposals between samples; dense holomorphic QGT.
    "tfim1d_n64_c": Workload("tfim1d_n64_c", "tfim", "chain", 64, 1.0, 1.0, 1, 1024, 16, 64,
                             "local", "c128"),
    # 1D TFIM chain L=20 after a quench to h=1 (J=1), complex RBM alpha=1,
    # 4096 samples (256 chains x 16), L proposals between samples.
    "tfim1d_n20_quench": Workload("tfim1d_n20_quench", "tfim", "chain", 20, 1.0, 1.0, 1, 256,
                                  16, 20, "local", "c128"),
}
