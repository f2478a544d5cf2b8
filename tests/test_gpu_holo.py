"""GPU-vs-oracle parity of the complex holomorphic RBM path (precision c128)
through the C ABI, on seeded synthetic inputs.

Bars:
  * Metropolis decisions, configurations and chain ends: bit-exact with the
    oracle's cached-tanh sampler (its smallest |u - |ratio|^2| must exceed
    1e-12 so no decision is ambiguous);
  * ln psi, local energies, Jacobian and force: within 1e-10 relative
    (ln psi's imaginary part compared modulo 2 pi);
  * SR directions and TDVP right-hand sides: the GPU's CG against the oracle's
    Cholesky solve of the same (G + eps I) x = f, within 1e-7 of |x| at a CG
    tolerance of 1e-11; the parameters after a step within 1e-8 of |theta|.
"""
import numpy as np
import pytest

import synth
from oracle import core, holo

pytestmark = pytest.mark.gpu

TFIM1D = synth.WORKLOADS["tfim1d_n10"].replace(precision="c128")


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible HIP device")
    return torch


def make_state(w, n_chains=None, params=None, **kw):
    _torch()
    from paper_2112_10526_amd.nqs import VMCState
    w2 = w.replace(**kw) if kw else w
    print(f"[case] {w2.name} L={w2.L} alpha={w2.alpha} prec={w2.precision} "
          f"chains={n_chains or w2.n_chains} S={w2.samples_per_chain}", flush=True)
    return VMCState.from_workload(w2, n_chains=n_chains, params=params), w2


def oracle_model(w, params):
    return (holo.RbmC(w.n_sites, w.n_hidden, params),
            core.Hamiltonian.tfim(w.n_sites, w.bonds(), w.J, w.h))


def rel_close(a, b, tol, scale=None):
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    s = np.maximum(np.abs(b), 1.0) if scale is None else scale
    err = np.abs(a - b) / s
    assert err.max() <= tol, f"max rel err {err.max():.3e} > {tol:.1e} at {int(err.argmax())}"


def wrap_close(a, b, tol):
    """ln psi: real parts within tol, imaginary parts within tol modulo 2 pi."""
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    rel_close(a.real, b.real, tol)
    d = np.angle(np.exp(1j * (a.imag - b.imag)))
    assert np.abs(d).max() <= tol * np.maximum(np.abs(b.imag), 1.0).max()


# ----------------------------------------------------------------------------
# sampler: one wave per chain, hidden units split 64 per lane slot
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("L,alpha,chains,S,sigma", [
    (10, 1, 16, 64, 0.3),     # M = 10: one hidden slot per lane
    (10, 1, 15, 16, 0.05),    # odd chain count
    (64, 2, 32, 4, 0.05),     # M = 128: two slots
    (20, 4, 24, 8, 0.1),      # M = 80: two slots, ragged
    (64, 4, 8, 2, 0.03),      # M = 256: four slots
    (64, 8, 8, 2, 0.02),      # M = 512: eight slots (the largest)
])
def test_sampler_bit_exact(L, alpha, chains, S, sigma):
    w = TFIM1D.replace(L=L, alpha=alpha, samples_per_chain=S, sweep_size=L, sigma=sigma)
    st, w = make_state(w, n_chains=chains)
    ch0 = st.get_chains()
    smp, acc, a = st.sample(log_accepts=True)
    rbm, _ = oracle_model(w, w.params())
    ref = holo.sample(rbm, ch0, S, w.sweep_size, w.chain_seed, 0, mode="cached",
                      log_accepts=True)
    assert ref.margins.min() > 1e-12
    np.testing.assert_array_equal(acc.cpu().numpy(), ref.accepts)
    np.testing.assert_array_equal(smp.cpu().numpy(), ref.samples)
    np.testing.assert_array_equal(st.get_chains(), ref.chains)
    assert abs(a - ref.n_accepted.sum() / ref.accepts.size) < 1e-15
    # the next call continues the same streams from the chain ends
    smp2, acc2, _ = st.sample(log_accepts=True)
    ref2 = holo.sample(rbm, ref.chains, S, w.sweep_size, w.chain_seed, S * w.sweep_size,
                       mode="cached", log_accepts=True)
    assert ref2.margins.min() > 1e-12
    np.testing.assert_array_equal(acc2.cpu().numpy(), ref2.accepts)
    np.testing.assert_array_equal(smp2.cpu().numpy(), ref2.samples)


def test_thermalize_and_discard_continue_the_streams():
    w = TFIM1D.replace(sigma=0.2, samples_per_chain=8)
    st, w = make_state(w)
    ch0 = st.get_chains()
    st.thermalize(3)
    smp, _, _ = st.sample(n_discard=2)
    rbm, _ = oracle_model(w, w.params())
    K = w.sweep_size
    t = holo.sample(rbm, ch0, 3, K, w.chain_seed, 0, mode="cached")
    d = holo.sample(rbm, t.chains, 2, K, w.chain_seed, 3 * K, mode="cached")
    ref = holo.sample(rbm, d.chains, 8, K, w.chain_seed, 5 * K, mode="cached")
    assert min(t.margins.min(), d.margins.min(), ref.margins.min()) > 1e-12
    np.testing.assert_array_equal(smp.cpu().numpy(), ref.samples)


# ----------------------------------------------------------------------------
# per-sample quantities
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("L,alpha,n,sigma", [(10, 1, 37, 0.3), (20, 2, 300, 0.2),
                                             (64, 1, 1000, 0.05), (64, 8, 129, 0.02)])
def test_log_psi_local_energy_jacobian(L, alpha, n, sigma):
    torch = _torch()
    w = TFIM1D.replace(L=L, alpha=alpha, sigma=sigma)
    st, w = make_state(w)
    s = synth.random_configs(n, w.n_sites, 11 + L)
    rbm, ham = oracle_model(w, w.params())
    sd = torch.from_numpy(s).cuda()
    wrap_close(st.log_psi(sd).cpu().numpy(), holo.log_psi(rbm, s), 1e-12)
    rel_close(st.local_energy(sd).cpu().numpy(), holo.local_energy(rbm, ham, s), 1e-10)
    rel_close(st.jacobian(sd).cpu().numpy(), holo.jacobian(rbm, s), 1e-12)


def test_empty_batches():
    torch = _torch()
    st, w = make_state(TFIM1D)
    s = torch.zeros((0, w.n_sites), dtype=torch.int8, device="cuda")
    assert st.local_energy(s).numel() == 0
    assert st.log_psi(s).numel() == 0


# ----------------------------------------------------------------------------
# estimators and the solve
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("L,alpha,chains,S", [(10, 1, 16, 64), (20, 2, 64, 16),
                                              (64, 1, 128, 8)])
def test_energy_force_and_sr_direction(L, alpha, chains, S):
    torch = _torch()
    w = TFIM1D.replace(L=L, alpha=alpha, samples_per_chain=S, sigma=0.1)
    st, w = make_state(w, n_chains=chains)
    s = synth.random_configs(chains * S, w.n_sites, 5 + L)
    st.load_samples(torch.from_numpy(s).cuda())
    E, g = st.expect_and_grad()
    rbm, ham = oracle_model(w, w.params())
    El = holo.local_energy(rbm, ham, s)
    O = holo.jacobian(rbm, s)
    ref = holo.energy_stats(El)
    assert abs(E["mean"] - ref["mean"].real) <= 1e-10 * max(abs(ref["mean"]), 1.0)
    assert abs(E["variance"] - ref["variance"]) <= 1e-9 * max(ref["variance"], 1.0)
    f = holo.force(O, El)
    rel_close(g.cpu().numpy(), f, 1e-10, scale=np.abs(f).max())
    eps, lr = 0.01, 0.05
    p0 = st.get_params()
    d, info = st.sr_update(diag_shift=eps, lr=lr, tol=1e-11, maxiter=4 * O.shape[1])
    x = holo.cholesky_solve(O, f, eps)
    assert info.converged
    rel_close(d.cpu().numpy(), x, 1e-7, scale=np.abs(x).max())
    rel_close(st.get_params(), p0 - lr * d.cpu().numpy(), 1e-14)


def test_vmc_step_matches_oracle_step():
    w = TFIM1D.replace(sigma=0.1, samples_per_chain=32)
    st, w = make_state(w)
    rbm, ham = oracle_model(w, w.params())
    ch0 = st.get_chains()
    rep = st.vmc_step(diag_shift=0.01, lr=0.05, tol=1e-11, maxiter=1000)
    new, chains, orep = holo.vmc_step(rbm, ham, ch0, w.samples_per_chain, w.sweep_size,
                                      w.chain_seed, 0, 0.01, 0.05, 1e-11, 1000)
    np.testing.assert_array_equal(st.get_chains(), chains)
    assert abs(rep.energy["mean"] - orep.energy["mean"].real) <= 1e-10 * abs(orep.energy["mean"])
    assert abs(rep.energy["acceptance"] - orep.acceptance) < 1e-15
    assert rep.sr.converged
    rel_close(st.get_params(), new.params, 1e-8, scale=np.abs(rbm.params).max())


@pytest.mark.parametrize("scheme", ["euler", "heun"])
@pytest.mark.parametrize("gamma", [-1j, -1.0])
def test_tdvp_step_matches_oracle_step(scheme, gamma):
    w = synth.WORKLOADS["tfim1d_n20_quench"].replace(L=12, n_chains=64, samples_per_chain=16,
                                                      sweep_size=12, sigma=0.1)
    st, w = make_state(w)
    rbm, ham = oracle_model(w, w.params())
    ch0 = st.get_chains()
    dt, eps = 0.01, 1e-3
    stages = st.tdvp_step(dt, gamma=gamma, scheme=scheme, diag_shift=eps, tol=1e-11,
                          maxiter=2000)
    new, chains, reps, used = holo.tdvp_step(rbm, ham, ch0, w.samples_per_chain, w.sweep_size,
                                             w.chain_seed, 0, dt, gamma, scheme, eps, 1e-11,
                                             2000)
    assert len(stages) == len(reps) == (2 if scheme == "heun" else 1)
    assert st.proposal_count == used
    np.testing.assert_array_equal(st.get_chains(), chains)
    for g, r in zip(stages, reps):
        assert g["solve"].converged
        assert abs(g["energy"]["mean"] - r.energy["mean"]) <= 1e-10 * abs(r.energy["mean"])
    rel_close(st.get_params(), new.params, 1e-8, scale=np.abs(rbm.params).max())


# ----------------------------------------------------------------------------
# what the complex path refuses
# ----------------------------------------------------------------------------
def test_complex_refusals():
    torch = _torch()
    from paper_2112_10526_amd._lib import NqsError
    from paper_2112_10526_amd.nqs import VMCState
    w = TFIM1D
    with pytest.raises(NqsError):  # exchange moves are not offered for complex models
        VMCState(model="tfim", n_sites=w.n_sites, bonds=w.bonds(), J=1.0, h=1.0,
                 n_hidden=w.n_hidden, precision="c128", rule="exchange", n_chains=4,
                 samples_per_chain=2, sweep_size=10, seed=1, params=w.params())
    with pytest.raises(NqsError):  # M above the sampler's 512 hidden units
        VMCState(model="tfim", n_sites=w.n_sites, bonds=w.bonds(), J=1.0, h=1.0,
                 n_hidden=520, precision="c128", n_chains=4, samples_per_chain=2,
                 sweep_size=10, seed=1)
    with pytest.raises(NqsError):  # TFIM only
        VMCState(model="heisenberg", n_sites=w.n_sites, bonds=w.bonds(), J=1.0,
                 n_hidden=w.n_hidden, precision="c128", n_chains=4, samples_per_chain=2,
                 sweep_size=10, seed=1, params=w.params())
    st, w = make_state(TFIM1D)
    s = torch.from_numpy(synth.random_configs(4, w.n_sites, 1)).cuda()
    with pytest.raises(NqsError):
        st.log_psi_vjp(s, torch.ones(4, dtype=torch.complex128, device="cuda"))
    with pytest.raises(NqsError):
        st.jacobian(s, center=True)
    real, _ = make_state(synth.WORKLOADS["tfim1d_n10"])
    with pytest.raises(NqsError):  # TDVP needs complex parameters
        real.tdvp_step(0.01)


def test_sampled_quench_follows_exact_dynamics():
    """The real-time example's quench at L = 12 on the GPU: SR at h = 1/2 gives
    the initial complex RBM (alpha = 1); TDVP Heun steps (dt = 0.01, 8192
    samples per evaluation) at h = 1.  Every 10 steps the GPU's parameters are
    evaluated exactly (all 4096 configurations through the oracle's ln psi)
    and compared with exp(-i H1 t)|psi_0> from the same initial state, so only
    the sampling noise of the equation of motion and the variational error
    remain: fidelity, sum_i <sigma^x_i> and the (conserved) energy."""
    import scipy.sparse.linalg as spla
    from oracle import exact
    from paper_2112_10526_amd.nqs import VMCState
    w = synth.WORKLOADS["tfim1d_n20_quench"].replace(L=12, sweep_size=12, n_chains=512)
    prep, _ = make_state(w.replace(h=0.5))
    prep.thermalize(50)
    for _ in range(200):
        prep.vmc_step(diag_shift=0.01, lr=0.02, tol=1e-6)
    st = VMCState.from_workload(w, params=prep.get_params())
    st.set_chains(prep.get_chains())
    N, M = w.n_sites, w.n_hidden
    ham = core.Hamiltonian.tfim(N, w.bonds(), w.J, w.h)
    H1 = exact.hamiltonian_matrix(ham)
    X = sum(exact.site_op(exact._X, i, N) for i in range(N))
    cfg = exact.all_configs(N)

    def state(p):
        lp = holo.log_psi(holo.RbmC(N, M, p), cfg)
        v = np.exp(lp - lp.real.max())
        return v / np.linalg.norm(v)

    psi0 = state(st.get_params())
    E0 = np.vdot(psi0, H1 @ psi0).real
    for k in range(1, 51):
        stages = st.tdvp_step(0.01, gamma=-1j, scheme="heun", diag_shift=1e-3, tol=1e-6)
        assert all(g["solve"].converged for g in stages)
        if k % 10 == 0:
            ref = spla.expm_multiply(-1j * H1 * (0.01 * k), psi0)
            v = state(st.get_params())
            fid = abs(np.vdot(ref, v)) ** 2
            dsx = np.vdot(v, X @ v).real - np.vdot(ref, X @ ref).real
            dE = np.vdot(v, H1 @ v).real - E0
            print(f"[quench] t={0.01 * k:.2f} fidelity={fid:.6f} dSx={dsx:+.4f} dE={dE:+.5f} "
                  f"(E0={E0:.5f})", flush=True)
            assert fid > 0.99 and abs(dsx) < 0.25 and abs(dE) < 0.01 * abs(E0)
