"""Symmetric RBM (the paper's RBMSymm): the oracle of the symmetric-model path.

TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline timing).  Nothing
here is imported by the product library.

What it follows (paper: table of models, "RBMSymm"; symmetric NQS section,
symmetric-RBM equation): a one-layer group-convolutional network whose alpha
features are aggregated by a product over the group,
    psi(s) = exp(a sum_k s_k) prod_{i < alpha, g in G} cosh f_g^(i)(s),
    f_g^(i)(s) = b_i + sum_k W_i[k] s[perm_g[k]],
so ln psi = a sum_k s_k + sum_{i,g} ln cosh f_g^(i); G is given as site
permutations (row 0 the identity; the rows must form a group).  The
visible-bias term is the group-invariant a sum_k s_k (one scalar a).

Parameters, packed: [a (1, if visible bias) | b (alpha, if hidden bias) |
W (alpha x N, row-major)].  The log-derivatives are the sums over the group
    O_a = sum_k s_k,  O_{b_i} = sum_g tanh f_g^(i),
    O_{W_i[k]} = sum_g tanh f_g^(i) s[perm_g[k]],
and the model equals a plain RBM with alpha |G| hidden units (hidden unit
i |G| + g has weights W_i scattered by perm_g, bias b_i, and every visible
bias a): `expand` writes that RBM out, so the plain RBM's sampler and local
energies serve here; it is pinned against the definition above.
Estimators (force, QGT, CG) are the plain RBM's (real parameters, 1/N_s).
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

from . import core


def check_group(perms) -> np.ndarray:
    """Rows are permutations of 0..N-1, row 0 is the identity, and the set is
    closed under composition; returns the table as int64."""
    P = np.asarray(perms, dtype=np.int64)
    if P.ndim != 2 or P.shape[0] < 1:
        raise ValueError("perms must be [G][N]")
    G, N = P.shape
    for g in range(G):
        if not np.array_equal(np.sort(P[g]), np.arange(N)):
            raise ValueError(f"row {g} is not a permutation")
    if not np.array_equal(P[0], np.arange(N)):
        raise ValueError("row 0 must be the identity")
    rows = {tuple(r) for r in P}
    if len(rows) != G:
        raise ValueError("repeated permutation")
    for g in range(G):
        for h in range(G):
            if tuple(P[g][P[h]]) not in rows:
                raise ValueError("the permutations do not form a group")
    return P


@dataclasses.dataclass
class RbmSymm:
    perms: np.ndarray   # [G][N]
    alpha: int
    params: np.ndarray
    visible_bias: bool = True
    hidden_bias: bool = True

    def __post_init__(self):
        self.perms = check_group(self.perms)
        self.params = np.ascontiguousarray(self.params, dtype=np.float64)
        if self.params.size != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters, got {self.params.size}")

    @property
    def N(self) -> int:
        return self.perms.shape[1]

    @property
    def G(self) -> int:
        return self.perms.shape[0]

    @property
    def n_params(self) -> int:
        return (1 if self.visible_bias else 0) + (self.alpha if self.hidden_bias else 0) \
            + self.alpha * self.N

    def parts(self):
        """(a, b [alpha], W [alpha, N]) with zeros for absent biases."""
        k, a, b = 0, 0.0, np.zeros(self.alpha)
        if self.visible_bias:
            a = self.params[0]
            k = 1
        if self.hidden_bias:
            b = self.params[k:k + self.alpha]
            k += self.alpha
        return a, b, self.params[k:].reshape(self.alpha, self.N)

    def with_params(self, p) -> "RbmSymm":
        return RbmSymm(self.perms, self.alpha, p, self.visible_bias, self.hidden_bias)


def _cfg(r: RbmSymm, s) -> np.ndarray:
    return np.asarray(s, dtype=np.float64).reshape(-1, r.N)


def features(r: RbmSymm, s) -> np.ndarray:
    """f[n, i, g] = b_i + sum_k W_i[k] s_n[perm_g[k]]."""
    s = _cfg(r, s)
    _, b, W = r.parts()
    sg = s[:, r.perms]                       # [n, G, N]: s_n[perm_g[k]]
    return np.einsum("ik,ngk->nig", W, sg) + b[None, :, None]


def log_psi(r: RbmSymm, s) -> np.ndarray:
    s = _cfg(r, s)
    a, _, _ = r.parts()
    return a * s.sum(axis=1) + np.log(np.cosh(features(r, s))).sum(axis=(1, 2))


def jacobian(r: RbmSymm, s) -> np.ndarray:
    """O[n, p] = d ln psi(s_n) / d theta_p in the packed layout."""
    s = _cfg(r, s)
    t = np.tanh(features(r, s))              # [n, alpha, G]
    cols = []
    if r.visible_bias:
        cols.append(s.sum(axis=1, keepdims=True))
    if r.hidden_bias:
        cols.append(t.sum(axis=2))
    cols.append(np.einsum("nig,ngk->nik", t, s[:, r.perms]).reshape(s.shape[0], -1))
    return np.concatenate(cols, axis=1)


def expand(r: RbmSymm) -> core.Rbm:
    """The equivalent plain RBM: hidden unit j = i |G| + g with
    W[j][perm_g[k]] = W_i[k], b_j = b_i, and visible biases all a."""
    a, b, W = r.parts()
    N, G, A = r.N, r.G, r.alpha
    Wf = np.zeros((A * G, N))
    for i in range(A):
        for g in range(G):
            Wf[i * G + g, r.perms[g]] = W[i]
    bf = np.repeat(b, G)
    af = np.full(N, a)
    return core.Rbm(N, A * G, np.concatenate([af, bf, Wf.ravel()]))


def sample(r: RbmSymm, chains, S: int, K: int, seed: int, prop_base: int, rule: str = "local",
           bonds=None, mode: str = "cached", log_accepts: bool = False):
    """Metropolis sampling of |psi|^2 with the plain RBM's sampler on expand(r)."""
    return core.sample(expand(r), chains, S, K, seed, prop_base, rule, bonds, mode=mode,
                       log_accepts=log_accepts)


def local_energy(r: RbmSymm, ham: core.Hamiltonian, s) -> np.ndarray:
    """E_loc(s) = sum_s' H(s, s') psi(s') / psi(s) from ln psi itself: the TFIM
    (diagonal J sum s_a s_b, single flips -h) and the Heisenberg model (diagonal
    J sum s_a s_b, exchanges of anti-aligned pairs 2J, times -1 across the two
    sublattices when Marshall labels are given)."""
    s = np.asarray(s, dtype=np.int8).reshape(-1, r.N)
    b = ham.bonds
    sd = s.astype(np.float64)
    E = ham.J * (sd[:, b[:, 0]] * sd[:, b[:, 1]]).sum(axis=1)
    lp = log_psi(r, s)
    if ham.kind == 0:      # TFIM
        for i in range(r.N):
            sp = s.copy()
            sp[:, i] = -sp[:, i]
            E = E - ham.h * np.exp(log_psi(r, sp) - lp)
    else:                  # Heisenberg
        sub = ham.sublattice
        for a_, b_ in b:
            anti = s[:, a_] != s[:, b_]
            if not anti.any():
                continue
            sp = s.copy()
            sp[:, [a_, b_]] = sp[:, [b_, a_]]
            sign = -1.0 if (sub is not None and sub[a_] != sub[b_]) else 1.0
            E = E + np.where(anti, 2.0 * ham.J * sign * np.exp(log_psi(r, sp) - lp), 0.0)
    return E


def solve_dense(O: np.ndarray, f: np.ndarray, diag_shift: float, tol: float,
                maxiter: Optional[int] = None):
    """(S + eps I) delta = f by CG on the dense S (QGTJacobianDense)."""
    S = core.qgt_dense(O) + diag_shift * np.eye(O.shape[1])
    if maxiter is None:
        maxiter = min(f.size, 10000)
    return core.cg(lambda v: S @ v, f, tol, maxiter)


def vmc_step(r: RbmSymm, ham: core.Hamiltonian, chains, S: int, K: int, seed: int,
             prop_base: int, diag_shift: float, lr: float, tol: float,
             maxiter: Optional[int] = None, rule: str = "local", mode: str = "cached"):
    """sample -> local energies -> force -> dense SR solve -> update."""
    res = sample(r, chains, S, K, seed, prop_base, rule, ham.bonds, mode=mode)
    flat = res.samples.reshape(-1, r.N)
    E = local_energy(r, ham, flat)
    O = jacobian(r, flat)
    f = core.force(O, E)
    delta, it, resid, _ = solve_dense(O, f, diag_shift, tol, maxiter)
    acc = res.n_accepted.sum() / (chains.shape[0] * S * K)
    rep = core.StepReport(core.energy_stats(E), f, delta, it, resid, acc, res.samples, E)
    return r.with_params(r.params - lr * delta), res.chains, rep


class ExactStateSymm:
    """Full-sum expectations over |psi(s)|^2 / Z (the paper's ExactState)."""

    def __init__(self, r: RbmSymm, ham: core.Hamiltonian):
        from . import exact
        self.r, self.ham = r, ham
        self.configs = exact.all_configs(r.N)
        lp = log_psi(r, self.configs)
        self.psi = np.exp(lp - lp.max())
        w = self.psi ** 2
        self.p = w / w.sum()
        self.H = exact.hamiltonian_matrix(ham)

    def energy(self) -> float:
        v = self.psi
        return float(v @ (self.H @ v) / (v @ v))

    def force(self) -> np.ndarray:
        O = jacobian(self.r, self.configs)
        E = (self.H @ self.psi) / self.psi
        p = self.p
        return 2.0 * (O - p @ O).T @ (p * (E - p @ E))
