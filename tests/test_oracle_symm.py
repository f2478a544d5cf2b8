"""Pins of the symmetric-RBM oracle (oracle/symm.py) against the definition,
the symmetry it encodes, finite differences and full enumeration."""
import numpy as np
import pytest

import synth
from oracle import core, exact, symm


def _model(perms, alpha, scale, seed, vb=True, hb=True):
    N = np.asarray(perms).shape[1]
    p = synth.symm_params(N, alpha, seed, scale, vb, hb)
    return symm.RbmSymm(perms, alpha, p, vb, hb)


GROUPS = {
    "chain8": synth.chain_translations(8),
    "square3": synth.square_translations(3),
    "swap4": np.array([[0, 1, 2, 3], [3, 1, 2, 0]]),  # the paper's four-site example
}


def test_translation_tables_are_groups():
    for name, g in GROUPS.items():
        symm.check_group(g)
    symm.check_group(synth.square_translations(4))
    with pytest.raises(ValueError):   # not closed: a lone translation by one site
        symm.check_group(np.array([[0, 1, 2, 3], [1, 2, 3, 0]]))
    with pytest.raises(ValueError):   # identity not first
        symm.check_group(np.array([[3, 1, 2, 0], [0, 1, 2, 3]]))
    with pytest.raises(ValueError):   # not a permutation
        symm.check_group(np.array([[0, 1, 2, 3], [0, 0, 2, 3]]))


@pytest.mark.parametrize("name", list(GROUPS))
def test_log_psi_is_invariant_under_the_group(name):
    perms = GROUPS[name]
    r = _model(perms, 2, 0.4, 1)
    s = synth.random_configs(50, r.N, 2)
    lp = symm.log_psi(r, s)
    for g in range(r.G):
        np.testing.assert_allclose(symm.log_psi(r, s[:, perms[g]]), lp, rtol=0, atol=1e-12)


def test_paper_example_swaps_first_and_last_site():
    r = _model(GROUPS["swap4"], 1, 0.5, 3)
    cfg = exact.all_configs(4)
    np.testing.assert_allclose(symm.log_psi(r, cfg), symm.log_psi(r, cfg[:, [3, 1, 2, 0]]),
                               atol=1e-13)
    # and a model that is not symmetric under it (a plain RBM) generally is not
    rbm = core.Rbm(4, 2, synth.rbm_params(4, 2, 4, 0.5))
    assert np.abs(core.log_psi(rbm, cfg) - core.log_psi(rbm, cfg[:, [3, 1, 2, 0]])).max() > 1e-3


@pytest.mark.parametrize("vb,hb", [(True, True), (False, True), (True, False)])
def test_expanded_rbm_equals_the_definition(vb, hb):
    r = _model(GROUPS["square3"], 3, 0.3, 5, vb, hb)
    s = synth.random_configs(40, r.N, 6)
    np.testing.assert_allclose(core.log_psi(symm.expand(r), s), symm.log_psi(r, s),
                               rtol=1e-13, atol=1e-12)


@pytest.mark.parametrize("vb,hb", [(True, True), (False, False)])
def test_jacobian_matches_finite_differences(vb, hb):
    r = _model(GROUPS["chain8"], 2, 0.3, 7, vb, hb)
    s = synth.random_configs(6, r.N, 8)
    O = symm.jacobian(r, s)
    h = 1e-6
    for k in range(r.n_params):
        e = np.zeros(r.n_params)
        e[k] = h
        d = (symm.log_psi(r.with_params(r.params + e), s) -
             symm.log_psi(r.with_params(r.params - e), s)) / (2 * h)
        np.testing.assert_allclose(O[:, k], d, rtol=1e-7, atol=1e-8)


def test_jacobian_is_the_tied_plain_jacobian():
    """O_sym = O_full T, T the derivative of the expansion (chain rule)."""
    r = _model(GROUPS["square3"], 2, 0.3, 9)
    s = synth.random_configs(20, r.N, 10)
    Of = core.jacobian(symm.expand(r), s)
    T = np.zeros((symm.expand(r).n_params, r.n_params))
    for k in range(r.n_params):   # expand is linear in the parameters
        e = np.zeros(r.n_params)
        e[k] = 1.0
        T[:, k] = symm.expand(r.with_params(e)).params
    np.testing.assert_allclose(Of @ T, symm.jacobian(r, s), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("kind", ["tfim", "heis"])
def test_local_energy_is_H_psi_over_psi(kind):
    perms = synth.chain_translations(8)
    r = _model(perms, 2, 0.3, 11)
    bonds = synth.chain_bonds(8)
    ham = (core.Hamiltonian.tfim(8, bonds, 1.0, 0.7) if kind == "tfim" else
           core.Hamiltonian.heisenberg(8, bonds, 1.0, synth.chain_sublattice(8)))
    ex = symm.ExactStateSymm(r, ham)
    E = symm.local_energy(r, ham, ex.configs)
    np.testing.assert_allclose(E, (ex.H @ ex.psi) / ex.psi, rtol=1e-10, atol=1e-10)
    # the plain RBM's local energies on the expanded model agree
    np.testing.assert_allclose(core.local_energy(symm.expand(r), ham, ex.configs), E,
                               rtol=1e-10, atol=1e-10)


def test_exact_force_is_finite_difference_of_energy():
    r = _model(synth.chain_translations(6), 2, 0.3, 12)
    ham = core.Hamiltonian.tfim(6, synth.chain_bonds(6), 1.0, 1.0)
    f = symm.ExactStateSymm(r, ham).force()
    h = 1e-5
    for k in range(r.n_params):
        e = np.zeros(r.n_params)
        e[k] = h
        ep = symm.ExactStateSymm(r.with_params(r.params + e), ham).energy()
        em = symm.ExactStateSymm(r.with_params(r.params - e), ham).energy()
        assert abs(f[k] - (ep - em) / (2 * h)) < 1e-6 * max(1.0, abs(f[k]))


def test_vmc_reaches_the_pfeuty_energy():
    """SR with the translation-symmetric RBM (alpha = 2, 23 parameters) on the
    periodic TFIM chain N = 10, J = h = 1: the closed-form ground energy."""
    N = 10
    r = _model(synth.chain_translations(N), 2, 0.01, 13)
    ham = core.Hamiltonian.tfim(N, synth.chain_bonds(N), 1.0, 1.0)
    chains = core.init_chains(N, 16, 13)
    res = symm.sample(r, chains, 10, N, 13, 0)   # thermalisation: 10 N proposals
    chains, prop = res.chains, 10 * N
    Es = []
    for _ in range(120):
        r, chains, rep = symm.vmc_step(r, ham, chains, 64, N, 13, prop, 0.01, 0.05, 1e-6)
        prop += 64 * N
        Es.append(rep.energy["mean"])
    e0 = exact.tfim_chain_ground_energy(N, 1.0, 1.0)
    assert abs(np.mean(Es[-20:]) - e0) < 2e-3 * abs(e0), (np.mean(Es[-20:]), e0)
