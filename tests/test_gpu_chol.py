"""The dense direct solve (nqs_set_dense_solver(NQS_SOLVER_CHOLESKY)) against the
oracle's Cholesky solve of the same shifted QGT system, for plain FP64 models,
symmetric models and complex models (through the real embedding), at sizes
below, at and across the 32-column panels: SR directions within 1e-10 of the
direction's largest entry.  A TDVP step with the direct solve matches the
oracle's step; a system that is not positive definite reports NQS_ENUMERIC.
"""
import numpy as np
import pytest

import synth
from oracle import core, holo, symm

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible HIP device")
    return torch


def rel_close(a, b, tol, scale):
    err = np.abs(np.asarray(a) - np.asarray(b)) / scale
    assert err.max() <= tol, f"max rel err {err.max():.3e} > {tol:.1e} at {int(err.argmax())}"


def plain_state(L, alpha, chains, S, solver="cholesky", precision="fp64"):
    _torch()
    from paper_2112_10526_amd.nqs import VMCState
    w = synth.WORKLOADS["tfim1d_n10"].replace(L=L, alpha=alpha, sweep_size=L, sigma=0.1,
                                             samples_per_chain=S, precision=precision)
    print(f"[case] chol plain L={L} alpha={alpha} P={w.n_params} Ns={chains * S}", flush=True)
    st = VMCState(model="tfim", n_sites=w.n_sites, bonds=w.bonds(), J=1.0, h=1.0,
                  n_hidden=w.n_hidden, precision=precision, n_chains=chains,
                  samples_per_chain=S, sweep_size=L, seed=2, qgt="jacobian_dense",
                  params=w.params(), dense_solver=solver)
    return st, w


@pytest.mark.parametrize("L,alpha,chains,S", [(4, 1, 16, 8), (10, 1, 16, 64), (9, 1, 16, 32),
                                              (20, 1, 64, 16), (12, 3, 64, 16)])
def test_plain_direction(L, alpha, chains, S):
    torch = _torch()
    st, w = plain_state(L, alpha, chains, S)
    s = synth.random_configs(chains * S, w.n_sites, 3 + L)
    st.load_samples(torch.from_numpy(s).cuda())
    st.expect_and_grad()
    d, info = st.sr_update(qgt="jacobian_dense", diag_shift=0.01, lr=0.05)
    assert info.converged and info.iterations == 0
    rbm = core.Rbm(w.n_sites, w.n_hidden, w.params())
    ham = core.Hamiltonian.tfim(w.n_sites, w.bonds(), 1.0, 1.0)
    O = core.jacobian(rbm, s)
    f = core.force(O, core.local_energy(rbm, ham, s))
    x = core.cholesky_solve(core.qgt_dense(O), f, 0.01)
    rel_close(d.cpu().numpy(), x, 1e-10, np.abs(x).max())


@pytest.mark.parametrize("lattice,side,alpha", [("chain", 10, 2), ("square", 10, 2)])
def test_symmetric_direction(lattice, side, alpha):
    torch = _torch()
    from paper_2112_10526_amd.nqs import VMCState
    chain = lattice == "chain"
    N = side if chain else side * side
    perms = synth.chain_translations(side) if chain else synth.square_translations(side)
    bonds = synth.chain_bonds(side) if chain else synth.square_bonds(side)
    p = synth.symm_params(N, alpha, 1, 0.1)
    print(f"[case] chol symm {lattice}{side} alpha={alpha}", flush=True)
    st = VMCState(model="tfim", n_sites=N, bonds=bonds, J=1.0, h=1.0, n_hidden=0, n_chains=64,
                  samples_per_chain=16, sweep_size=N, seed=2, params=p, symmetries=perms,
                  alpha=alpha, dense_solver="cholesky")
    s = synth.random_configs(64 * 16, N, 5)
    st.load_samples(torch.from_numpy(s).cuda())
    st.expect_and_grad()
    d, info = st.sr_update(diag_shift=0.01, lr=0.05)
    assert info.converged
    r = symm.RbmSymm(perms, alpha, p)
    ham = core.Hamiltonian.tfim(N, bonds, 1.0, 1.0)
    O = symm.jacobian(r, s)
    f = core.force(O, symm.local_energy(r, ham, s))
    x = core.cholesky_solve(core.qgt_dense(O), f, 0.01)
    rel_close(d.cpu().numpy(), x, 1e-10, np.abs(x).max())


def complex_state(L, alpha, chains, S, sigma=0.1):
    _torch()
    from paper_2112_10526_amd.nqs import VMCState
    w = synth.WORKLOADS["tfim1d_n20_quench"].replace(L=L, alpha=alpha, sweep_size=L,
                                                      n_chains=chains, samples_per_chain=S,
                                                      sigma=sigma)
    print(f"[case] chol complex L={L} alpha={alpha} P={w.n_params}", flush=True)
    st = VMCState(model="tfim", n_sites=w.n_sites, bonds=w.bonds(), J=w.J, h=w.h,
                  n_hidden=w.n_hidden, precision="c128", n_chains=chains, samples_per_chain=S,
                  sweep_size=L, seed=w.chain_seed, params=w.params(), dense_solver="cholesky")
    return st, w


@pytest.mark.parametrize("L,alpha", [(10, 1), (20, 1)])
def test_complex_direction(L, alpha):
    torch = _torch()
    st, w = complex_state(L, alpha, 64, 16)
    s = synth.random_configs(64 * 16, w.n_sites, 7)
    st.load_samples(torch.from_numpy(s).cuda())
    st.expect_and_grad()
    d, info = st.sr_update(diag_shift=0.01, lr=0.05)
    assert info.converged
    rbm = holo.RbmC(w.n_sites, w.n_hidden, w.params())
    ham = core.Hamiltonian.tfim(w.n_sites, w.bonds(), w.J, w.h)
    O = holo.jacobian(rbm, s)
    f = holo.force(O, holo.local_energy(rbm, ham, s))
    x = holo.cholesky_solve(O, f, 0.01)
    rel_close(d.cpu().numpy(), x, 1e-10, np.abs(x).max())


def test_tdvp_step_with_the_direct_solve():
    st, w = complex_state(12, 1, 64, 16)
    rbm = holo.RbmC(w.n_sites, w.n_hidden, w.params())
    ham = core.Hamiltonian.tfim(w.n_sites, w.bonds(), w.J, w.h)
    ch0 = st.get_chains()
    stages = st.tdvp_step(0.01, gamma=-1j, scheme="heun", diag_shift=1e-3)
    new, chains, reps, _ = holo.tdvp_step(rbm, ham, ch0, w.samples_per_chain, w.sweep_size,
                                          w.chain_seed, 0, 0.01, -1j, "heun", 1e-3, 1e-13, 5000)
    np.testing.assert_array_equal(st.get_chains(), chains)
    assert all(g["solve"].iterations == 0 for g in stages)
    rel_close(st.get_params(), new.params, 1e-9, np.abs(rbm.params).max())


def test_not_positive_definite_is_reported():
    torch = _torch()
    from paper_2112_10526_amd._lib import NqsError
    st, w = plain_state(10, 1, 4, 8)
    s = np.ones((32, w.n_sites), dtype=np.int8)  # identical samples: S = 0 exactly
    st.load_samples(torch.from_numpy(s).cuda())
    st.expect_and_grad()
    with pytest.raises(NqsError) as e:
        st.sr_update(qgt="jacobian_dense", diag_shift=0.0, lr=0.05)
    assert e.value.status == 4  # NQS_ENUMERIC


def test_direct_solve_needs_the_fp64_gram():
    from paper_2112_10526_amd._lib import NqsError
    with pytest.raises(NqsError):
        plain_state(10, 1, 16, 8, precision="fp32")
