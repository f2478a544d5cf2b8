"""Pins of the complex (holomorphic) RBM oracle against what the paper and the
mathematics fix: brute-force marginalisation over the hidden units, the
Cauchy-Riemann relations (finite differences in the real and imaginary
directions), E_loc = (H psi)/psi with Kronecker-product Hamiltonians, the exact
force = the Wirtinger derivative dE/dtheta* of the exact energy, the QGT = its
definition from amplitude derivatives (QGT equation), detailed balance of the
sampler, complex CG against a direct solve, the real embedding of the Hermitian
system, VMC convergence to the free-fermion energy, and the TDVP: energy
conservation for real time and agreement with exact evolution where the
ansatz spans the Hilbert space."""
import itertools

import numpy as np
import pytest

import synth
from oracle import core, exact, holo


def _rbm(N, M, scale, seed):
    rng = np.random.default_rng(seed)
    P = N + M + M * N
    return holo.RbmC(N, M, scale * (rng.normal(size=P) + 1j * rng.normal(size=P)))


def _chain(N):
    return np.array([(i, (i + 1) % N) for i in range(N)], dtype=np.int32)


def test_log_psi_is_marginal_over_hidden_units():
    """psi(s) = sum_h exp(a.s + b.h + h^T W s) over h in {+-1}^M equals
    e^{a.s} prod_j 2 cosh(theta_j) (RBM of the table of models)."""
    N, M = 4, 3
    r = _rbm(N, M, 0.4, 1)
    a, b, W = r.params[:N], r.params[N:N + M], r.params[N + M:].reshape(M, N)
    cfg = exact.all_configs(N)
    lp = holo.log_psi(r, cfg)
    brute = []
    for s in cfg:
        tot = 0.0
        for h in itertools.product((1, -1), repeat=M):
            h = np.array(h)
            tot += np.exp(a @ s + b @ h + h @ (W @ s))
        brute.append(tot)
    brute = np.array(brute)
    ratio = np.exp(lp - lp[0]) / (brute / brute[0])
    np.testing.assert_allclose(ratio, 1.0, atol=1e-12)


def test_jacobian_cauchy_riemann():
    """d ln psi / d Re theta_k = O_k and d ln psi / d Im theta_k = i O_k."""
    N, M = 5, 4
    r = _rbm(N, M, 0.2, 2)
    s = synth.random_configs(6, N, 3)
    O = holo.jacobian(r, s)
    h = 1e-6
    for k in range(r.n_params):
        for step, fac in ((h, 1.0), (1j * h, 1j)):
            e = np.zeros(r.n_params, dtype=np.complex128)
            e[k] = step
            d = (holo.log_psi(r.with_params(r.params + e), s) -
                 holo.log_psi(r.with_params(r.params - e), s)) / (2 * h)
            np.testing.assert_allclose(d, fac * O[:, k], atol=2e-9, rtol=0)


@pytest.mark.parametrize("kind", ["tfim", "heis"])
def test_local_energy_is_H_psi_over_psi(kind):
    N, M = 6, 4
    r = _rbm(N, M, 0.3, 4)
    bonds = _chain(N)
    if kind == "tfim":
        ham = core.Hamiltonian.tfim(N, bonds, 1.0, 0.7)
    else:
        ham = core.Hamiltonian.heisenberg(N, bonds, 1.0, (np.arange(N) % 2).astype(np.int8))
    ex = holo.ExactStateC(r, ham)
    E = holo.local_energy(r, ham, ex.configs)
    np.testing.assert_allclose(E, ex.local_energies(), rtol=1e-12, atol=1e-12)


def test_exact_force_is_wirtinger_derivative_of_energy():
    """f~ = dE/dtheta* = (dE/dRe theta + i dE/dIm theta) / 2 for a holomorphic ansatz
    (complex co-gradient equation)."""
    N, M = 4, 2
    r = _rbm(N, M, 0.3, 5)
    ham = core.Hamiltonian.tfim(N, _chain(N), 1.0, 0.9)
    f = holo.ExactStateC(r, ham).force()
    h = 1e-6
    fd = np.zeros(r.n_params, dtype=np.complex128)
    for k in range(r.n_params):
        g = []
        for step in (h, 1j * h):
            e = np.zeros(r.n_params, dtype=np.complex128)
            e[k] = step
            ep = holo.ExactStateC(r.with_params(r.params + e), ham).energy()
            em = holo.ExactStateC(r.with_params(r.params - e), ham).energy()
            g.append((ep - em) / (2 * h))
        fd[k] = 0.5 * (g[0] + 1j * g[1])
    np.testing.assert_allclose(f, fd, atol=1e-8)


def test_qgt_matches_definition_from_amplitude_derivatives():
    """G_ij = <d_i psi|d_j psi>/<psi|psi> - <d_i psi|psi><psi|d_j psi>/<psi|psi>^2
    (QGT equation) with d_j psi by central differences of the amplitude vector."""
    N, M = 4, 2
    r = _rbm(N, M, 0.3, 6)
    ham = core.Hamiltonian.tfim(N, _chain(N), 1.0, 1.0)
    cfg = exact.all_configs(N)

    def amp(p):
        return np.exp(holo.log_psi(r.with_params(p), cfg))

    psi = amp(r.params)
    h = 1e-6
    D = np.zeros((cfg.shape[0], r.n_params), dtype=np.complex128)
    for k in range(r.n_params):
        e = np.zeros(r.n_params, dtype=np.complex128)
        e[k] = h
        D[:, k] = (amp(r.params + e) - amp(r.params - e)) / (2 * h)
    nn = np.vdot(psi, psi)
    G = D.conj().T @ D / nn - np.outer(D.conj().T @ psi, psi.conj() @ D) / nn ** 2
    np.testing.assert_allclose(holo.ExactStateC(r, ham).qgt(), G, atol=1e-8)


def test_mc_estimators_reduce_to_exact_sums_on_all_configs():
    """The sample estimators of force and QGT weighted by |psi|^2 over every
    configuration equal the exact sums; on sampled batches they agree within
    statistical error."""
    N, M = 6, 3
    r = _rbm(N, M, 0.25, 7)
    ham = core.Hamiltonian.tfim(N, _chain(N), 1.0, 1.0)
    ex = holo.ExactStateC(r, ham)
    chains = core.init_chains(N, 64, 11)
    res = holo.sample(r, chains, 0, N, 11, 0)
    res = holo.sample(r, res.chains, 256, N, 11, 64 * N, mode="cached")
    flat = res.samples.reshape(-1, N)
    E = holo.local_energy(r, ham, flat)
    st = holo.energy_stats(E)
    assert abs(st["mean"].real - ex.energy()) < 5 * st["error"] * 3  # chains are correlated
    O = holo.jacobian(r, flat)
    G = holo.qgt_dense(O)
    assert np.abs(G - ex.qgt()).max() < 0.05 * np.abs(ex.qgt()).max()
    assert np.allclose(G, G.conj().T)


def test_sampler_detailed_balance_chi2():
    N, M = 5, 3
    r = _rbm(N, M, 0.5, 8)
    ex = holo.ExactStateC(r, core.Hamiltonian.tfim(N, _chain(N), 1.0, 1.0))
    chains = core.init_chains(N, 32, 21)
    res = holo.sample(r, chains, 2000, 3, 21, 0, mode="cached")
    flat = res.samples[:, 200:].reshape(-1, N)
    idx = ((flat < 0).astype(np.int64) * (1 << (N - 1 - np.arange(N)))).sum(axis=1)
    counts = np.bincount(idx, minlength=2 ** N)
    expct = ex.p * flat.shape[0]
    chi2 = ((counts - expct) ** 2 / expct).sum()
    # 31 degrees of freedom; correlated samples inflate chi2 a little
    assert chi2 < 120, chi2


def test_sampler_modes_agree_bit_for_bit():
    N, M = 8, 8
    r = _rbm(N, M, 0.3, 9)
    chains = core.init_chains(N, 16, 31)
    a = holo.sample(r, chains, 6, N, 31, 0, mode="definition", log_accepts=True)
    b = holo.sample(r, chains, 6, N, 31, 0, mode="cached", log_accepts=True)
    np.testing.assert_array_equal(a.samples, b.samples)
    np.testing.assert_array_equal(a.accepts, b.accepts)
    assert a.margins.min() > 1e-12


def test_complex_cg_matches_direct_solve_and_real_embedding():
    """CG on the Hermitian system equals numpy's solve; the same system written
    over the reals, [[Re G, -Im G], [Im G, Re G]] [Re x; Im x] = [Re f; Im f], is
    symmetric positive definite and its CG iterates are the complex ones."""
    rng = np.random.default_rng(10)
    O = rng.normal(size=(300, 40)) + 1j * rng.normal(size=(300, 40))
    f = rng.normal(size=40) + 1j * rng.normal(size=40)
    eps = 0.05
    G = holo.qgt_dense(O) + eps * np.eye(40)
    x, it, res, conv = holo.cg(lambda v: G @ v, f, 1e-12, 500)
    assert conv
    np.testing.assert_allclose(x, np.linalg.solve(G, f), rtol=1e-9, atol=1e-11)
    n = O.shape[0]
    dO = (O - O.mean(axis=0)) / np.sqrt(n)
    Y = np.block([[dO.real, -dO.imag], [dO.imag, dO.real]])
    R = Y.T @ Y + eps * np.eye(80)
    np.testing.assert_allclose(R, np.block([[G.real, -G.imag], [G.imag, G.real]]), atol=1e-12)
    xr, itr, _, _ = core.cg(lambda v: R @ v, np.concatenate([f.real, f.imag]), 1e-12, 500)
    assert itr == it
    np.testing.assert_allclose(xr[:40] + 1j * xr[40:], x, rtol=1e-9, atol=1e-11)


def test_vmc_converges_to_free_fermion_energy():
    """Complex RBM, periodic TFIM chain N = 10, J = h = 1: SR with the dense
    holomorphic QGT reaches the closed-form ground energy."""
    N, M = 10, 10
    rng = np.random.default_rng(12)
    P = N + M + M * N
    r = holo.RbmC(N, M, 0.01 * (rng.normal(size=P) + 1j * rng.normal(size=P)))
    ham = core.Hamiltonian.tfim(N, _chain(N), 1.0, 1.0)
    chains = core.init_chains(N, 16, 13)
    prop = 0
    res = holo.sample(r, chains, 0, 10 * N, 13, prop)
    chains = res.chains
    prop += 100 * N
    Es = []
    for it in range(150):
        r, chains, rep = holo.vmc_step(r, ham, chains, 64, N, 13, prop, 0.01, 0.05, 1e-6)
        prop += 64 * N
        Es.append(rep.energy["mean"].real)
    e0 = exact.tfim_chain_ground_energy(N, 1.0, 1.0)
    assert abs(np.mean(Es[-20:]) - e0) < 2e-3 * abs(e0), (np.mean(Es[-20:]), e0)


def test_exact_tdvp_conserves_energy_in_real_time():
    """gamma = -i: dE/dt = 2 Re(f^H theta_dot) = 2 Re(-i f^H G^-1 f) = 0, so with
    Heun steps the energy drifts only at second order in dt (halving dt cuts
    the drift by about four); gamma = -1 (imaginary time) lowers the energy."""
    N, M = 6, 2  # fewer parameters than states: G is invertible
    r = _rbm(N, M, 0.3, 14)
    ham = core.Hamiltonian.tfim(N, _chain(N), 1.0, 1.0)
    E0 = holo.ExactStateC(r, ham).energy()
    drift = []
    for dt in (0.01, 0.005):
        q = r
        for _ in range(round(0.1 / dt)):
            q = holo.exact_tdvp_step(q, ham, dt, -1j, "heun")
        drift.append(abs(holo.ExactStateC(q, ham).energy() - E0))
    assert drift[1] < 1e-4 and drift[0] / drift[1] > 3.0, drift
    q = r
    for _ in range(10):
        q = holo.exact_tdvp_step(q, ham, 0.01, -1.0, "heun")
    assert holo.ExactStateC(q, ham).energy() < E0 - 1e-3


def test_exact_tdvp_follows_exact_evolution():
    """With 16 hidden units on 4 sites the tangent space covers the state
    space, so the TDVP trajectory (exact expectations, Heun) follows
    exp(-iHt)|psi_0>: fidelity and <sigma_x> at t = 0.1."""
    import scipy.linalg as sla
    N, M = 4, 16
    r = _rbm(N, M, 0.2, 15)
    ham = core.Hamiltonian.tfim(N, _chain(N), 1.0, 1.0)
    H = exact.hamiltonian_matrix(ham).toarray()
    cfg = exact.all_configs(N)
    psi0 = np.exp(holo.log_psi(r, cfg))
    psi0 /= np.linalg.norm(psi0)
    dt, steps = 0.002, 50
    for _ in range(steps):
        r = holo.exact_tdvp_step(r, ham, dt, -1j, "heun", diag_shift=1e-9)
    psi = np.exp(holo.log_psi(r, cfg))
    psi /= np.linalg.norm(psi)
    ref = sla.expm(-1j * H * dt * steps) @ psi0
    fid = abs(np.vdot(ref, psi)) ** 2
    assert fid > 1 - 1e-5, fid
    X = sum(exact.site_op(exact._X, i, N) for i in range(N)).toarray()
    assert abs(np.vdot(psi, X @ psi).real - np.vdot(ref, X @ ref).real) < 1e-3


def test_exact_tdvp_quench_tracks_exact_dynamics():
    """The real-time example's quench at L = 8: the complex RBM (alpha = 1) is
    brought to the h = 1/2 ground state by imaginary-time TDVP (exact
    expectations), then evolved in real time with h = 1 by Heun steps of
    dt = 0.01.  Against exp(-i H1 t)|psi_0> (sparse matrix exponential of the
    exact Hamiltonian applied to the same initial state): fidelity above
    0.999, <sum sigma^x> within 0.01 and the energy conserved to 5e-4
    relative up to t = 0.6."""
    import scipy.sparse.linalg as spla
    N, M = 8, 8
    rng = np.random.default_rng(3)
    P = N + M + M * N
    r = holo.RbmC(N, M, 0.05 * (rng.normal(size=P) + 1j * rng.normal(size=P)))
    h0 = core.Hamiltonian.tfim(N, _chain(N), 1.0, 0.5)
    h1 = core.Hamiltonian.tfim(N, _chain(N), 1.0, 1.0)
    for _ in range(60):
        r = holo.exact_tdvp_step(r, h0, 0.2, -1.0, "euler", diag_shift=1e-4)
    e0 = spla.eigsh(exact.hamiltonian_matrix(h0), k=1, which="SA")[0][0]
    assert abs(holo.ExactStateC(r, h0).energy() - e0) < 1e-4 * abs(e0)
    H1 = exact.hamiltonian_matrix(h1)
    X = sum(exact.site_op(exact._X, i, N) for i in range(N))
    cfg = exact.all_configs(N)

    def state(q):
        v = np.exp(holo.log_psi(q, cfg))
        return v / np.linalg.norm(v)

    psi0 = state(r)
    E0 = np.vdot(psi0, H1 @ psi0).real
    for k in range(1, 61):
        r = holo.exact_tdvp_step(r, h1, 0.01, -1j, "heun", diag_shift=1e-5)
        if k % 20 == 0:
            ref = spla.expm_multiply(-1j * H1 * (0.01 * k), psi0)
            v = state(r)
            assert abs(np.vdot(ref, v)) ** 2 > 0.999, k
            assert abs(np.vdot(v, X @ v).real - np.vdot(ref, X @ ref).real) < 0.01, k
            assert abs(np.vdot(v, H1 @ v).real - E0) < 5e-4 * abs(E0), k
