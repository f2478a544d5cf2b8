"""GPU-vs-oracle parity of the symmetric RBM (nqs_set_rbm_symm) through the C ABI.

Bars: sampling bit-exact (oracle margins above 1e-12); FP64 ln psi and local
energies within 1e-10 relative, the FP64 Jacobian within 1e-12; force within
1e-10 of its largest entry; SR directions against the oracle's Cholesky solve
within 1e-7 at CG tol 1e-11; a VMC step's parameters within 1e-9; FP32 and
BF16 forms: local energies within 1e-4 relative on the same batch, the
Jacobian within 1e-5 (FP32) and 3e-4 (BF16).
"""
import numpy as np
import pytest

import synth
from oracle import core, symm

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible HIP device")
    return torch


CASES = {
    # name: (model, lattice side, group, alpha, rule)
    "tfim_chain10": ("tfim", 10, "chain", 2, "local"),
    "tfim_square4": ("tfim", 4, "square", 3, "local"),
    "tfim_square10": ("tfim", 10, "square", 2, "local"),
    "heis_chain16": ("heisenberg", 16, "chain", 1, "exchange"),
}


def build(name, precision="fp64", n_chains=32, S=8, sigma=0.05, seed=1, vb=True, hb=True):
    _torch()
    from paper_2112_10526_amd.nqs import VMCState
    model, L, lat, alpha, rule = CASES[name]
    N = L if lat == "chain" else L * L
    bonds = synth.chain_bonds(L) if lat == "chain" else synth.square_bonds(L)
    perms = synth.chain_translations(L) if lat == "chain" else synth.square_translations(L)
    sub = None
    if model == "heisenberg":
        sub = synth.chain_sublattice(L) if lat == "chain" else synth.square_sublattice(L)
        ham = core.Hamiltonian.heisenberg(N, bonds, 1.0, sub)
    else:
        ham = core.Hamiltonian.tfim(N, bonds, 1.0, 1.0)
    p = synth.symm_params(N, alpha, seed, sigma, vb, hb)
    print(f"[case] symm {name} prec={precision} chains={n_chains} S={S} vb={vb} hb={hb}",
          flush=True)
    st = VMCState(model=model, n_sites=N, bonds=bonds, J=1.0, h=1.0, sublattice=sub,
                  n_hidden=0, visible_bias=vb, hidden_bias=hb, precision=precision, rule=rule,
                  n_chains=n_chains, samples_per_chain=S, sweep_size=N, seed=2,
                  total_sz_zero=(model == "heisenberg"), params=p, symmetries=perms,
                  alpha=alpha)
    return st, symm.RbmSymm(perms, alpha, p, vb, hb), ham


def rel_close(a, b, tol, scale=None):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    s = np.maximum(np.abs(b), 1.0) if scale is None else scale
    err = np.abs(a - b) / s
    assert err.max() <= tol, f"max rel err {err.max():.3e} > {tol:.1e} at {int(err.argmax())}"


@pytest.mark.parametrize("name,chains", [("tfim_chain10", 16), ("tfim_square4", 33),
                                         ("tfim_square10", 64), ("heis_chain16", 32)])
def test_sampler_bit_exact(name, chains):
    st, r, ham = build(name, n_chains=chains, S=4, sigma=0.1)
    ch0 = st.get_chains()
    smp, acc, _ = st.sample(log_accepts=True)
    rule = CASES[name][4]
    ref = symm.sample(r, ch0, 4, r.N, 2, 0, rule=rule, bonds=ham.bonds, log_accepts=True)
    assert ref.margins.min() > 1e-12
    np.testing.assert_array_equal(acc.cpu().numpy(), ref.accepts)
    np.testing.assert_array_equal(smp.cpu().numpy(), ref.samples)
    np.testing.assert_array_equal(st.get_chains(), ref.chains)


@pytest.mark.parametrize("name,vb,hb", [("tfim_chain10", True, True), ("tfim_square4", False, True),
                                        ("tfim_square10", True, False),
                                        ("heis_chain16", True, True)])
def test_log_psi_local_energy_jacobian(name, vb, hb):
    torch = _torch()
    st, r, ham = build(name, sigma=0.2, vb=vb, hb=hb)
    s = synth.random_configs(300, r.N, 7)
    sd = torch.from_numpy(s).cuda()
    rel_close(st.log_psi(sd).cpu().numpy(), symm.log_psi(r, s), 1e-12)
    rel_close(st.local_energy(sd).cpu().numpy(), symm.local_energy(r, ham, s), 1e-10)
    J = st.jacobian(sd).cpu().numpy()
    rel_close(J, symm.jacobian(r, s), 1e-12)
    # centred: (O - mean O) / sqrt(n)
    Oc = symm.jacobian(r, s)
    Oc = (Oc - Oc.mean(axis=0)) / np.sqrt(s.shape[0])
    rel_close(st.jacobian(sd, center=True).cpu().numpy(), Oc, 1e-12)


def test_group_invariance_on_the_gpu():
    torch = _torch()
    st, r, _ = build("tfim_square4", sigma=0.3)
    s = synth.random_configs(64, r.N, 9)
    lp = st.log_psi(torch.from_numpy(s).cuda()).cpu().numpy()
    for g in range(r.G):
        lg = st.log_psi(torch.from_numpy(np.ascontiguousarray(s[:, r.perms[g]])).cuda())
        np.testing.assert_allclose(lg.cpu().numpy(), lp, rtol=0, atol=1e-12)


@pytest.mark.parametrize("name", ["tfim_chain10", "tfim_square10", "heis_chain16"])
def test_force_and_sr_direction(name):
    torch = _torch()
    st, r, ham = build(name, n_chains=64, S=16, sigma=0.1)
    s = synth.random_configs(64 * 16, r.N, 11)
    if name.startswith("heis"):
        s = synth.sz0_configs(64 * 16, r.N, 11)
    st.load_samples(torch.from_numpy(s).cuda())
    E, g = st.expect_and_grad()
    El = symm.local_energy(r, ham, s)
    O = symm.jacobian(r, s)
    ref = core.energy_stats(El)
    assert abs(E["mean"] - ref["mean"]) <= 1e-10 * max(abs(ref["mean"]), 1.0)
    f = core.force(O, El)
    rel_close(g.cpu().numpy(), f, 1e-10, scale=np.abs(f).max())
    eps, lr = 0.01, 0.05
    p0 = st.get_params()
    d, info = st.sr_update(diag_shift=eps, lr=lr, tol=1e-11, maxiter=10 * r.n_params)
    assert info.converged
    x = core.cholesky_solve(core.qgt_dense(O), f, eps)
    rel_close(d.cpu().numpy(), x, 1e-7, scale=np.abs(x).max())
    rel_close(st.get_params(), p0 - lr * d.cpu().numpy(), 1e-14)


def test_vmc_steps_match_the_oracle():
    st, r, ham = build("tfim_chain10", n_chains=16, S=32, sigma=0.05)
    chains = st.get_chains()
    prop = 0
    for _ in range(3):
        rep = st.vmc_step(diag_shift=0.01, lr=0.05, tol=1e-11, maxiter=1000)
        r, chains, orep = symm.vmc_step(r, ham, chains, 32, r.N, 2, prop, 0.01, 0.05, 1e-11, 1000)
        prop += 32 * r.N
        np.testing.assert_array_equal(st.get_chains(), chains)
        assert abs(rep.energy["mean"] - orep.energy["mean"]) <= 1e-10 * abs(orep.energy["mean"])
        assert rep.sr.converged
        rel_close(st.get_params(), r.params, 1e-9, scale=np.abs(r.params).max())


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_precision_forms_local_energies(precision):
    torch = _torch()
    st, r, ham = build("tfim_square10", precision=precision, n_chains=64, S=4, sigma=0.05)
    s = synth.random_configs(512, r.N, 13)
    sd = torch.from_numpy(s).cuda()
    rel_close(st.local_energy(sd).cpu().numpy(), symm.local_energy(r, ham, s), 1e-4)
    # the symmetric Jacobian from the form's FP32 activations: FP32 theta and tanh
    # (1e-5); the BF16 form's theta comes from the two-term BF16 split, about
    # 2^-16 relative per activation, and each entry sums |G| = 100 of them (3e-4)
    rel_close(st.jacobian(sd).cpu().numpy(), symm.jacobian(r, s),
              1e-5 if precision == "fp32" else 3e-4)
    rep = st.vmc_step(diag_shift=0.01, lr=0.01, tol=1e-6, maxiter=5000)
    print(f"[sr] {rep.sr}", flush=True)
    assert rep.sr.converged and np.isfinite(rep.energy["mean"])


def test_symmetric_refusals():
    torch = _torch()
    from paper_2112_10526_amd._lib import NqsError
    from paper_2112_10526_amd.nqs import VMCState
    N = 6
    common = dict(model="tfim", n_sites=N, bonds=synth.chain_bonds(N), J=1.0, h=1.0, n_hidden=0,
                  n_chains=4, samples_per_chain=2, sweep_size=N, seed=1, alpha=1)
    with pytest.raises(NqsError):  # a lone translation is not a group
        VMCState(symmetries=np.array([np.arange(N), (np.arange(N) + 1) % N]), **common)
    with pytest.raises(NqsError):  # identity not first
        VMCState(symmetries=synth.chain_translations(N)[::-1].copy(), **common)
    with pytest.raises(NqsError):  # complex parameters
        VMCState(symmetries=synth.chain_translations(N), precision="c128", **common)
    st = VMCState(symmetries=synth.chain_translations(N), params=synth.symm_params(N, 1, 1),
                  **common)
    assert st.n_params == 1 + 1 + N
    s = torch.from_numpy(synth.random_configs(4, N, 1)).cuda()
    with pytest.raises(NqsError):
        st.log_psi_vjp(s, torch.ones(4, dtype=torch.float64, device="cuda"))
    st.sample()
    st.expect_and_grad()
    import ctypes
    from paper_2112_10526_amd import _lib
    info = _lib.NqsSrInfo()
    assert st.lib.nqs_sr_update(st.ctx, _lib.QGTS["onthefly"], 0.01, 0.01, 1e-6, 0, None,
                                ctypes.byref(info)) == _lib.NQS_EINVAL
