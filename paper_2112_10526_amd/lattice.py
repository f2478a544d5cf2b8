"""Problem definitions a caller of the library needs to set up a run: bond lists
of periodic chains and square lattices, Marshall sublattice labels, and
initial RBM parameters.  None of the method's arithmetic lives here.

Conventions (paper, section on Hilbert spaces and graphs): the periodic chain
has bonds (i, i+1 mod n); the periodic L x L square lattice, site x + L y,
has bonds (x,y)-(x+1,y) and (x,y)-(x,y+1), each listed once (L >= 3).
Parameters use the packed layout of the C boundary,
[a (n_sites) | b (n_hidden) | W (n_hidden x n_sites, row-major)].
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

__all__ = ["chain_bonds", "square_bonds", "chain_sublattice", "square_sublattice",
           "init_params", "RunSpec"]


def chain_bonds(n: int) -> np.ndarray:
    if n < 3:
        raise ValueError("a periodic chain needs at least 3 sites")
    i = np.arange(n, dtype=np.int32)
    return np.ascontiguousarray(np.stack([i, (i + 1) % n], axis=1), dtype=np.int32)


def square_bonds(L: int) -> np.ndarray:
    if L < 3:
        raise ValueError("a periodic square lattice needs L >= 3")
    x = np.tile(np.arange(L), L)
    y = np.repeat(np.arange(L), L)
    s = x + L * y
    right = (x + 1) % L + L * y
    up = x + L * ((y + 1) % L)
    out = np.empty((2 * L * L, 2), dtype=np.int32)
    out[0::2, 0] = s
    out[0::2, 1] = right
    out[1::2, 0] = s
    out[1::2, 1] = up
    return out


def chain_sublattice(n: int) -> np.ndarray:
    return (np.arange(n) % 2).astype(np.int8)


def square_sublattice(L: int) -> np.ndarray:
    k = np.arange(L * L)
    return ((k % L + k // L) % 2).astype(np.int8)


def init_params(n_sites: int, n_hidden: int, seed: int, sigma: float = 0.01,
                visible_bias: bool = True, hidden_bias: bool = True) -> np.ndarray:
    """Parameters drawn i.i.d. from a normal distribution with standard
    deviation ``sigma`` (numpy's PCG64 generator seeded with ``seed``)."""
    P = (n_sites if visible_bias else 0) + (n_hidden if hidden_bias else 0) + n_sites * n_hidden
    return np.random.default_rng(seed).normal(0.0, sigma, size=P).astype(np.float64)


@dataclasses.dataclass(frozen=True)
class RunSpec:
    """Everything ``VMCState.from_workload`` reads to build one run."""
    model: str             # "tfim" or "heisenberg"
    lattice: str           # "chain" or "square"
    L: int
    J: float
    h: float
    alpha: int
    n_chains: int
    samples_per_chain: int
    sweep_size: int
    rule: str              # "local" or "exchange"
    precision: str
    param_seed: int = 1
    chain_seed: int = 2
    sigma: float = 0.01
    marshall: bool = False
    total_sz_zero: bool = False

    @property
    def n_sites(self) -> int:
        return self.L if self.lattice == "chain" else self.L * self.L

    @property
    def n_hidden(self) -> int:
        return self.alpha * self.n_sites

    @property
    def n_samples(self) -> int:
        return self.n_chains * self.samples_per_chain

    def bonds(self) -> np.ndarray:
        return chain_bonds(self.L) if self.lattice == "chain" else square_bonds(self.L)

    def sublattice(self) -> Optional[np.ndarray]:
        if not self.marshall:
            return None
        return chain_sublattice(self.L) if self.lattice == "chain" else square_sublattice(self.L)

    def params(self) -> np.ndarray:
        return init_params(self.n_sites, self.n_hidden, self.param_seed, self.sigma)
