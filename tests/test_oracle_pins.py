"""Pins for the FP64 oracle: every oracle function is checked here against
something other than itself -- a value the paper prints, a closed form, an
invariant, a library routine, or brute force on tiny inputs.

Pin map (oracle function -> pins):
  philox4x32_10 ............ rocRAND's Philox4x32-10 engine (library routine);
                             uniformity of the derived site index and u
  tfim / heisenberg matrix . paper's printed sigma^x algebra example; trace
                             identities; Pfeuty closed form (TFIM chain);
                             h = 0, J = 0 and large-h limits (square lattice);
                             singlet / 4-site ring closed forms (Heisenberg);
                             Marshall rotation preserves the spectrum and makes
                             the ground state sign-free
  log_psi .................. brute-force marginalisation over hidden units;
                             W = 0 product form
  local_energy ............. (H psi)(s) / psi(s) with the Kronecker-product H,
                             for every configuration
  jacobian ................. central finite differences of log_psi
  force .................... finite-difference gradient of the exact energy;
                             Monte Carlo estimate within 5 sigma of enumeration
  qgt_dense / qgt_matvec ... numpy.cov (biased) of the log-derivatives; Monte
                             Carlo estimate on exact draws within 5 sigma of the
                             enumerated QGT, which is pinned to the QGT
                             definition from wave-function derivatives
  cg / cholesky_solve ...... numpy.linalg.solve
  sample ................... zero parameters accept every move; detailed
                             balance (chi^2 against |psi|^2); definition and
                             cached modes give the same decisions
  init_chains .............. spin balance; exact zero magnetisation; uniform
                             placement
  vmc_step ................. the 1D chain N=10 converges towards the Pfeuty
                             ground energy
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import synth
from oracle import core, exact

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


# ----------------------------------------------------------------------------
# Philox
# ----------------------------------------------------------------------------
@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND reference")
    exe = str(tmp_path_factory.mktemp("philox") / "philox_ref")
    subprocess.run([hipcc, "-O1", "-o", exe, os.path.join(ROOT, "tests", "rocrand_philox_ref.cpp")],
                   check=True, capture_output=True)
    return exe


def test_philox_matches_rocrand(rocrand_ref, oracle_lib):
    rng = np.random.default_rng(7)
    cases = [(0, 0, 0, 0)]
    for _ in range(300):
        cases.append((int(rng.integers(0, 2**63)), int(rng.integers(0, 2**32)),
                      int(rng.integers(0, 4)), int(rng.integers(0, 2**40))))
    # rocRAND takes the offset in words (4 per draw), so p < 2^62 here.
    cases.append((2**64 - 1, 2**32 - 1, 3, 2**62 - 1))
    # rocRAND: key = seed, counter = (offset/4 lo, hi, subsequence lo, hi);
    # the oracle's draw for proposal p of chain g with tag t uses counter
    # (p lo, p hi, g, t), i.e. subsequence = g | t << 32.
    lines = "".join(f"{seed} {g | (t << 32)} {p}\n" for seed, g, t, p in cases)
    out = subprocess.run([rocrand_ref], input=lines, capture_output=True, text=True,
                         check=True).stdout.split("\n")
    for (seed, g, t, p), line in zip(cases, out):
        ref = [int(x) for x in line.split()]
        got = core.philox([p & 0xFFFFFFFF, p >> 32, g, t], seed)
        assert list(got) == ref, (seed, g, t, p)


def test_philox_site_and_uniform_statistics(oracle_lib):
    # The derived site index must be uniform on [0, N) and u uniform on [0, 1):
    # replay the oracle's own mapping through the zero-parameter sampler (every
    # move accepted), which exposes the site stream as the flip positions.
    N, C, S, K = 7, 64, 50, 1
    rbm = core.Rbm(N, 3, np.zeros(synth.n_params(N, 3)))
    chains = np.ones((C, N), dtype=np.int8)
    res = core.sample(rbm, chains, S, K, seed=11, prop_base=0)
    prev = np.concatenate([chains[:, None, :], res.samples[:, :-1, :]], axis=1)
    flips = np.argmax(prev != res.samples, axis=2).ravel()
    counts = np.bincount(flips, minlength=N)
    expected = flips.size / N
    chi2 = ((counts - expected) ** 2 / expected).sum()
    assert chi2 < 30.0  # 6 dof; p ~ 4e-5


# ----------------------------------------------------------------------------
# Hamiltonian matrices, ED and closed forms
# ----------------------------------------------------------------------------
def test_paper_operator_algebra_example():
    ref = np.loadtxt(os.path.join(ROOT, "tests", "golden", "paper_sigmax_square.txt"))
    X0 = exact.site_op(exact._X, 0, 2)
    X1 = exact.site_op(exact._X, 1, 2)
    op = (X0 + X1) @ (X0 + X1)
    np.testing.assert_array_equal(op.toarray().real, ref)
    np.testing.assert_array_equal((2 * (X0 @ X1) + 2 * exact.sp.identity(4)).toarray().real, ref)


@pytest.mark.parametrize("lattice,L", [("chain", 5), ("chain", 8), ("square", 3), ("square", 4)])
def test_bond_lists(lattice, L):
    b = synth.chain_bonds(L) if lattice == "chain" else synth.square_bonds(L)
    N = L if lattice == "chain" else L * L
    deg = np.bincount(b.ravel(), minlength=N)
    assert (deg == (2 if lattice == "chain" else 4)).all()
    pairs = {tuple(sorted(p)) for p in b.tolist()}
    assert len(pairs) == len(b)  # no bond listed twice
    assert len(b) == (N if lattice == "chain" else 2 * N)


@pytest.mark.parametrize("lattice,L", [("chain", 6), ("square", 3)])
def test_trace_identities(lattice, L):
    N = L if lattice == "chain" else L * L
    b = synth.chain_bonds(L) if lattice == "chain" else synth.square_bonds(L)
    J, h = 0.7, 1.3
    H = exact.tfim_matrix(N, b, J, h)
    dim = 2 ** N
    assert abs(H.diagonal().sum()) < 1e-9
    # Pauli strings are trace-orthogonal: Tr H^2 / 2^N = sum of squared coefficients.
    assert np.isclose((H.multiply(H)).sum() / dim, len(b) * J * J + N * h * h)
    Hh = exact.heisenberg_matrix(N, b, J)
    assert abs(Hh.diagonal().sum()) < 1e-9
    assert np.isclose((Hh.multiply(Hh)).sum() / dim, 3 * len(b) * J * J)


@pytest.mark.parametrize("N", [6, 8, 10, 12])
@pytest.mark.parametrize("h", [0.5, 1.0, 3.0])
def test_tfim_chain_matches_pfeuty(N, h):
    H = exact.tfim_matrix(N, synth.chain_bonds(N), 1.0, h)
    e0 = exact.ground_energy(H)[0]
    assert abs(e0 - exact.tfim_chain_ground_energy(N, 1.0, h)) < 1e-9


def test_tfim_chain_closed_form_special_value():
    # J = h = 1: E0 = -2 / sin(pi / 2N)
    for N in (8, 10, 12):
        assert np.isclose(exact.tfim_chain_ground_energy(N, 1, 1), -2 / np.sin(np.pi / (2 * N)),
                          rtol=1e-13)


def test_tfim_square_limits():
    # h = 0, bipartite 4x4: Neel state, E0 = -J * n_bonds.
    b4 = synth.square_bonds(4)
    assert np.isclose(exact.ground_energy(exact.tfim_matrix(16, b4, 1.0, 0.0))[0], -len(b4))
    # J = 0: E0 = -h N.
    b3 = synth.square_bonds(3)
    assert np.isclose(exact.ground_energy(exact.tfim_matrix(9, b3, 0.0, 2.0))[0], -18.0)
    # Large h on 4x4 (no loops of three bonds, so no third-order term):
    # E0 = -hN - n_b J^2 / (4h) + O(J^4/h^3); the residual must fall as h^-3.
    res = []
    for h in (20.0, 40.0):
        e0 = exact.ground_energy(exact.tfim_matrix(16, b4, 1.0, h))[0]
        res.append(e0 - (-h * 16 - len(b4) / (4 * h)))
    assert abs(res[1]) < 3e-4
    assert 6.0 < res[0] / res[1] < 10.0


def test_heisenberg_closed_forms():
    # Two sites, one bond: sigma.sigma has singlet eigenvalue -3.
    H2 = exact.heisenberg_matrix(2, np.array([[0, 1]]), 1.0)
    assert np.isclose(exact.ground_energy(H2)[0], -3.0)
    # 4-site ring: E0 = -2 J in spin-1/2 units, i.e. -8 J with Pauli matrices.
    H4 = exact.heisenberg_matrix(4, synth.chain_bonds(4), 1.0)
    assert np.isclose(exact.ground_energy(H4)[0], -8.0)


@pytest.mark.parametrize("N", [6, 8])
def test_marshall_rotation(N):
    b = synth.chain_bonds(N)
    H = exact.heisenberg_matrix(N, b, 1.0).toarray()
    Hm = exact.heisenberg_matrix(N, b, 1.0, synth.chain_sublattice(N)).toarray()
    np.testing.assert_allclose(np.linalg.eigvalsh(H), np.linalg.eigvalsh(Hm), atol=1e-10)
    # Rotated operator is stoquastic: off-diagonal elements <= 0, and its
    # ground state (zero magnetisation sector) has one sign.
    off = Hm - np.diag(np.diag(Hm))
    assert off.max() <= 1e-12
    mask = exact.sz0_mask(N)
    w, v = np.linalg.eigh(Hm[np.ix_(mask, mask)])
    g = v[:, 0] * np.sign(v[np.argmax(np.abs(v[:, 0])), 0])
    assert g.min() > -1e-10


# ----------------------------------------------------------------------------
# RBM log-amplitude and derivatives
# ----------------------------------------------------------------------------
def test_log_psi_is_marginal_over_hidden_units(oracle_lib):
    # An RBM amplitude is the Boltzmann weight summed over hidden units:
    # sum_{h in {+-1}^M} exp(a.s + h.(W s + b)) = 2^M psi(s).
    N, M = 5, 6
    rng = np.random.default_rng(3)
    p = rng.normal(0, 0.4, synth.n_params(N, M))
    rbm = core.Rbm(N, M, p)
    a, b, W = p[:N], p[N:N + M], p[N + M:].reshape(M, N)
    hs = exact.all_configs(M).astype(float)
    cfg = exact.all_configs(N)
    brute = []
    for s in cfg.astype(float):
        z = np.exp(a @ s + hs @ (W @ s + b)).sum()
        brute.append(np.log(z) - M * np.log(2.0))
    np.testing.assert_allclose(core.log_psi(rbm, cfg), brute, rtol=0, atol=1e-12)


def test_log_psi_product_state(oracle_lib):
    N, M = 6, 4
    a = np.linspace(-0.3, 0.4, N)
    b = np.linspace(0.1, 0.5, M)
    rbm = core.Rbm(N, M, np.concatenate([a, b, np.zeros(M * N)]))
    cfg = exact.all_configs(N)
    np.testing.assert_allclose(core.log_psi(rbm, cfg),
                               cfg @ a + np.log(np.cosh(b)).sum(), atol=1e-13)


@pytest.mark.parametrize("vb,hb", [(True, True), (False, True), (True, False)])
def test_jacobian_finite_differences(oracle_lib, vb, hb):
    N, M = 6, 5
    rng = np.random.default_rng(5)
    P = synth.n_params(N, M, vb, hb)
    rbm = core.Rbm(N, M, rng.normal(0, 0.3, P), vb, hb)
    s = synth.random_configs(7, N, 9)
    O = core.jacobian(rbm, s)
    eps = 1e-5
    fd = np.zeros_like(O)
    for k in range(P):
        pp = rbm.params.copy(); pp[k] += eps
        pm = rbm.params.copy(); pm[k] -= eps
        fd[:, k] = (core.log_psi(rbm.with_params(pp), s) - core.log_psi(rbm.with_params(pm), s)) / (2 * eps)
    np.testing.assert_allclose(O, fd, atol=1e-9)


# ----------------------------------------------------------------------------
# Local energies
# ----------------------------------------------------------------------------
def _hams(N, L=None):
    out = [("tfim_chain", core.Hamiltonian.tfim(N, synth.chain_bonds(N), 1.0, 1.3)),
           ("heis_chain", core.Hamiltonian.heisenberg(N, synth.chain_bonds(N), 1.0)),
           ("heis_chain_marshall", core.Hamiltonian.heisenberg(N, synth.chain_bonds(N), 0.8,
                                                               synth.chain_sublattice(N)))]
    return out


@pytest.mark.parametrize("which", [0, 1, 2])
def test_local_energy_matches_dense_hamiltonian(oracle_lib, which):
    N, M = 8, 8
    name, ham = _hams(N)[which]
    rbm = core.Rbm(N, M, synth.rbm_params(N, M, 4, sigma=0.3))
    es = exact.ExactState(rbm, ham)
    E = core.local_energy(rbm, ham, es.configs)
    np.testing.assert_allclose(E, es.local_energies(), rtol=1e-11, atol=1e-11)


def test_local_energy_tfim_square(oracle_lib):
    L = 3
    ham = core.Hamiltonian.tfim(9, synth.square_bonds(L), 1.0, 3.044)
    rbm = core.Rbm(9, 18, synth.rbm_params(9, 18, 2, sigma=0.2))
    es = exact.ExactState(rbm, ham)
    E = core.local_energy(rbm, ham, es.configs)
    np.testing.assert_allclose(E, es.local_energies(), rtol=1e-11, atol=1e-11)
    assert np.isclose(es.expectation_of(E), es.energy(), rtol=1e-12)


def test_zero_params_local_energy(oracle_lib):
    # psi uniform: E(s) = J sum_b s_a s_b - h N exactly.
    L = 10
    N = L * L
    b = synth.square_bonds(L)
    rbm = core.Rbm(N, 2 * N, np.zeros(synth.n_params(N, 2 * N)))
    ham = core.Hamiltonian.tfim(N, b, 1.0, 3.044)
    s = synth.random_configs(16, N, 1)
    diag = (s[:, b[:, 0]].astype(int) * s[:, b[:, 1]]).sum(axis=1)
    np.testing.assert_allclose(core.local_energy(rbm, ham, s), diag - 3.044 * N, atol=1e-12)


def test_product_state_closed_forms(oracle_lib):
    # W = 0, b = 0: <s_i> = tanh 2a_i, <H> = J sum_b tanh2a tanh2a - h sum 1/cosh 2a,
    # QGT a-block = diag(1/cosh^2 2a), O_b = O_W = 0.
    N, M = 8, 8
    a = np.linspace(-0.4, 0.35, N)
    rbm = core.Rbm(N, M, np.concatenate([a, np.zeros(M + M * N)]))
    b = synth.chain_bonds(N)
    ham = core.Hamiltonian.tfim(N, b, 1.0, 0.9)
    es = exact.ExactState(rbm, ham)
    t2 = np.tanh(2 * a)
    ref = (t2[b[:, 0]] * t2[b[:, 1]]).sum() - 0.9 * (1 / np.cosh(2 * a)).sum()
    assert np.isclose(es.energy(), ref, rtol=1e-13)
    G = es.qgt()
    np.testing.assert_allclose(G[:N, :N], np.diag(1 / np.cosh(2 * a) ** 2), atol=1e-13)
    assert np.abs(G[N:, :]).max() < 1e-14


# ----------------------------------------------------------------------------
# Force and QGT
# ----------------------------------------------------------------------------
def _exact_energy(rbm, H):
    v = np.exp(core.log_psi(rbm, exact.all_configs(rbm.N)))
    return v @ (H @ v) / (v @ v)


def test_exact_force_is_energy_gradient(oracle_lib):
    N, M = 6, 6
    rbm = core.Rbm(N, M, synth.rbm_params(N, M, 8, sigma=0.25))
    ham = core.Hamiltonian.tfim(N, synth.chain_bonds(N), 1.0, 0.7)
    H = exact.hamiltonian_matrix(ham)
    f = exact.ExactState(rbm, ham).force()
    eps = 1e-6
    fd = np.zeros(rbm.n_params)
    for k in range(rbm.n_params):
        pp = rbm.params.copy(); pp[k] += eps
        pm = rbm.params.copy(); pm[k] -= eps
        fd[k] = (_exact_energy(rbm.with_params(pp), H) - _exact_energy(rbm.with_params(pm), H)) / (2 * eps)
    np.testing.assert_allclose(f, fd, atol=2e-8)


def test_qgt_matches_definition(oracle_lib):
    # G_ij = <d_i psi|d_j psi>/<psi|psi> - <d_i psi|psi><psi|d_j psi>/<psi|psi>^2
    # with derivatives of the full amplitude vector taken by finite differences.
    N, M = 5, 4
    rbm = core.Rbm(N, M, synth.rbm_params(N, M, 3, sigma=0.3))
    ham = core.Hamiltonian.tfim(N, synth.chain_bonds(N), 1.0, 1.0)
    cfg = exact.all_configs(N)
    psi = np.exp(core.log_psi(rbm, cfg))
    eps = 1e-6
    D = np.zeros((psi.size, rbm.n_params))
    for k in range(rbm.n_params):
        pp = rbm.params.copy(); pp[k] += eps
        pm = rbm.params.copy(); pm[k] -= eps
        D[:, k] = (np.exp(core.log_psi(rbm.with_params(pp), cfg))
                   - np.exp(core.log_psi(rbm.with_params(pm), cfg))) / (2 * eps)
    n2 = psi @ psi
    G_def = D.T @ D / n2 - np.outer(D.T @ psi, psi @ D) / n2 ** 2
    np.testing.assert_allclose(exact.ExactState(rbm, ham).qgt(), G_def, atol=1e-8)


def test_qgt_onthefly_equals_dense_and_cg_solves(oracle_lib):
    N, M = 8, 16
    rbm = core.Rbm(N, M, synth.rbm_params(N, M, 5, sigma=0.2))
    s = synth.random_configs(300, N, 6)
    O = core.jacobian(rbm, s)
    rng = np.random.default_rng(0)
    v = rng.normal(size=rbm.n_params)
    S = core.qgt_dense(O)
    np.testing.assert_allclose(core.qgt_matvec(O, v, 0.01), S @ v + 0.01 * v, atol=1e-12)
    E = rng.normal(size=300)
    f = core.force(O, E)
    x, it, res, conv = core.cg(lambda u: core.qgt_matvec(O, u, 0.01), f, 1e-10, 5000)
    assert conv
    ref = np.linalg.solve(S + 0.01 * np.eye(S.shape[0]), f)
    np.testing.assert_allclose(x, ref, atol=1e-7 * np.abs(ref).max())
    np.testing.assert_allclose(core.cholesky_solve(S, f, 0.01), ref, atol=1e-9 * np.abs(ref).max())


def test_qgt_estimators_are_the_sample_covariance(oracle_lib):
    """qgt_dense is the biased (1/N_s) sample covariance of the log-derivatives
    (numpy.cov with bias=True, a library routine), and qgt_matvec applies it."""
    N, M = 6, 9
    rbm = core.Rbm(N, M, synth.rbm_params(N, M, 2, sigma=0.3))
    s = synth.random_configs(257, N, 3)
    O = core.jacobian(rbm, s)
    C = np.cov(O.T, bias=True)
    np.testing.assert_allclose(core.qgt_dense(O), C, rtol=0, atol=1e-13)
    v = np.random.default_rng(4).normal(size=rbm.n_params)
    np.testing.assert_allclose(core.qgt_matvec(O, v, 0.03), C @ v + 0.03 * v, rtol=0, atol=1e-12)


def test_qgt_monte_carlo_estimate_matches_enumeration(oracle_lib):
    """The estimator on independent draws from |psi|^2 / Z (drawn by enumeration,
    so no Markov chain is involved) agrees with the exact QGT of the full sum
    within 5 standard errors, entry by entry, and so does its product with a
    vector; dropping the centring or a factor would miss by many errors."""
    N, M = 8, 8
    rbm = core.Rbm(N, M, synth.rbm_params(N, M, 6, sigma=0.3))
    ham = core.Hamiltonian.tfim(N, synth.chain_bonds(N), 1.0, 1.0)
    es = exact.ExactState(rbm, ham)
    n = 40000
    idx = np.random.default_rng(8).choice(es.p.size, size=n, p=es.p)
    O = core.jacobian(rbm, es.configs[idx])
    S = core.qgt_dense(O)
    G = es.qgt()
    dO = O - O.mean(axis=0)
    se = np.sqrt(np.einsum("ki,kj->ij", dO ** 2, dO ** 2) / n - S ** 2) / np.sqrt(n)
    z = np.abs(S - G) / (se + 1e-15)
    assert (z < 5).mean() > 0.995, np.sort(z.ravel())[-10:]
    v = np.random.default_rng(9).normal(size=rbm.n_params)
    Gv = core.qgt_matvec(O, v, 0.0)
    t = dO @ v
    se_v = np.sqrt(((dO * t[:, None]) ** 2).mean(axis=0) - Gv ** 2) / np.sqrt(n)
    assert (np.abs(Gv - G @ v) < 5 * se_v + 1e-12).mean() > 0.99
    # the uncentred second moment is far outside the errors (the centring matters)
    assert np.median(np.abs(O.T @ O / n - G) / (se + 1e-15)) > 20


def test_cg_stopping_rule(oracle_lib):
    A = np.diag(np.arange(1.0, 41.0))
    f = np.ones(40)
    x, it, res, conv = core.cg(lambda u: A @ u, f, 1e-6, 1000)
    assert conv and res <= 1e-6 and it <= 40
    r = f - A @ x
    assert np.linalg.norm(r) <= 1e-6 * np.linalg.norm(f) * 1.0001
    x1, it1, res1, conv1 = core.cg(lambda u: A @ u, f, 1e-6, 1)
    assert it1 == 1 and not conv1


# ----------------------------------------------------------------------------
# Sampler and chains
# ----------------------------------------------------------------------------
def test_zero_params_accept_everything(oracle_lib):
    N, C, S, K = 12, 8, 20, 5
    rbm = core.Rbm(N, 6, np.zeros(synth.n_params(N, 6)))
    ch = core.init_chains(N, C, seed=3)
    res = core.sample(rbm, ch, S, K, seed=4, prop_base=100, log_accepts=True)
    assert res.accepts.all()
    assert (res.n_accepted == S * K).all()
    # Replaying the site stream reproduces every recorded sample.
    s = ch.copy().astype(int)
    for q in range(S * K):
        for c in range(C):
            x = core.philox([(100 + q) & 0xFFFFFFFF, (100 + q) >> 32, c, 0], 4)
            i = (int(x[0]) * N) >> 32
            s[c, i] = -s[c, i]
        if (q + 1) % K == 0:
            np.testing.assert_array_equal(res.samples[:, (q + 1) // K - 1], s)


@pytest.mark.parametrize("rule", ["local", "exchange"])
def test_definition_and_cached_modes_agree(oracle_lib, rule):
    L = 4
    N = L * L
    rbm = core.Rbm(N, 2 * N, synth.rbm_params(N, 2 * N, 1, sigma=0.1))
    b = synth.square_bonds(L)
    ch = core.init_chains(N, 32, seed=9, total_sz_zero=(rule == "exchange"))
    r0 = core.sample(rbm, ch, 3, N, 9, 0, rule, b, mode="definition", log_accepts=True)
    r1 = core.sample(rbm, ch, 3, N, 9, 0, rule, b, mode="cached", log_accepts=True)
    assert r0.margins.min() > 1e-12
    np.testing.assert_array_equal(r0.accepts, r1.accepts)
    np.testing.assert_array_equal(r0.samples, r1.samples)
    if rule == "exchange":
        assert (r0.samples.astype(int).sum(axis=2) == 0).all()


@pytest.mark.parametrize("rule", ["local", "exchange"])
def test_detailed_balance(oracle_lib, rule):
    # Many independent chains, each run for 100 N proposals, then one sample per
    # chain: the histogram must follow |psi|^2 / Z (chi^2 with dof = states - 1).
    N, M = 6, 6
    rbm = core.Rbm(N, M, synth.rbm_params(N, M, 12, sigma=0.3))
    b = synth.chain_bonds(N)
    sz0 = rule == "exchange"
    ch = core.init_chains(N, 8192, seed=5, total_sz_zero=sz0)
    res = core.sample(rbm, ch, 1, 100 * N, 21, 0, rule, b, mode="cached")
    flat = res.samples.reshape(-1, N)
    idx = ((1 - flat.astype(int)) // 2) @ (1 << (N - 1 - np.arange(N)))
    ham = core.Hamiltonian.heisenberg(N, b, 1.0)
    es = exact.ExactState(rbm, ham, sz0=sz0)
    counts = np.bincount(idx, minlength=2 ** N)
    assert counts[~es.mask].sum() == 0
    counts = counts[es.mask]
    expct = es.p[es.mask] * flat.shape[0]
    chi2 = ((counts - expct) ** 2 / expct).sum()
    dof = es.mask.sum() - 1
    assert chi2 < dof + 5 * np.sqrt(2 * dof), (chi2, dof)


def test_init_chains(oracle_lib):
    N, C = 100, 512
    s = core.init_chains(N, C, seed=2)
    assert set(np.unique(s)) <= {-1, 1}
    m = s.astype(int).mean()
    assert abs(m) < 4 / np.sqrt(N * C)
    z = core.init_chains(16, 4000, seed=3, total_sz_zero=True)
    assert (z.astype(int).sum(axis=1) == 0).all()
    up = (z > 0).mean(axis=0)  # each site up with probability 1/2
    assert np.abs(up - 0.5).max() < 5 * 0.5 / np.sqrt(4000)
    # different chain offsets continue the same stream
    np.testing.assert_array_equal(core.init_chains(N, 4, 2, chain_offset=10),
                                  s[10:14])


# ----------------------------------------------------------------------------
# Monte Carlo estimates vs enumeration, and a small VMC run
# ----------------------------------------------------------------------------
def test_mc_estimates_match_enumeration(oracle_lib):
    N, M = 8, 8
    rbm = core.Rbm(N, M, synth.rbm_params(N, M, 6, sigma=0.3))
    ham = core.Hamiltonian.tfim(N, synth.chain_bonds(N), 1.0, 1.0)
    es = exact.ExactState(rbm, ham)
    ch = core.init_chains(N, 256, seed=1)
    core.sample(rbm, ch, 1, 50 * N, 1, 0)  # warm the stream (not used)
    th = core.sample(rbm, ch, 1, 20 * N, 1, 0)
    res = core.sample(rbm, th.chains, 16, 2 * N, 1, 20 * N)
    flat = res.samples.reshape(-1, N)
    E = core.local_energy(rbm, ham, flat)
    st = core.energy_stats(E)
    assert abs(st["mean"] - es.energy()) < 5 * st["error"] * 2  # x2 for autocorrelation
    O = core.jacobian(rbm, flat)
    f = core.force(O, E)
    fe = es.force()
    # per-component standard error of 2 Cov(O, E)
    dE = E - E.mean()
    se = 2 * np.sqrt(((O - O.mean(0)) * dE[:, None]).var(axis=0) / E.size)
    assert (np.abs(f - fe) < 10 * se + 1e-12).mean() > 0.99


@pytest.mark.slow
def test_vmc_converges_tfim_chain(oracle_lib):
    w = synth.WORKLOADS["tfim1d_n10"]
    N, M = w.n_sites, w.n_hidden
    rbm = core.Rbm(N, M, w.params())
    ham = core.Hamiltonian.tfim(N, w.bonds(), w.J, w.h)
    ch = core.init_chains(N, w.n_chains, w.chain_seed)
    prop = 0
    th = core.sample(rbm, ch, 1, 100 * w.sweep_size, w.chain_seed, prop, mode="cached")
    ch, prop = th.chains, prop + 100 * w.sweep_size
    energies = []
    for step in range(150):
        rbm, ch, rep = core.vmc_step(rbm, ham, ch, w.samples_per_chain, w.sweep_size,
                                     w.chain_seed, prop, "local", w.diag_shift, 0.05,
                                     w.cg_tol)
        prop += w.samples_per_chain * w.sweep_size
        energies.append(rep.energy["mean"])
    e0 = exact.tfim_chain_ground_energy(N, 1.0, 1.0)
    assert abs(np.mean(energies[-20:]) - e0) < 0.003 * abs(e0)
