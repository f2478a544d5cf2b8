"""SR directions at the full shapes of the differentiation-form and precision-form
workloads, checked against the oracle's own QGT product on the same batch.

Property checked (no full oracle solve at these sizes): the direction d returned
by the library satisfies the oracle's system (S + eps I) d = f up to
    |(S + eps I) d - f| <= 2 tol |f| + e |S + eps I|_2 |d| + |g - f|,
where tol is the CG tolerance (the CG recurrence residual is below tol |f|; the
true residual of the computed iterate may differ from it by the same amount
again), e |S + eps I|_2 |d| bounds the rounding of the form's operator, and
g - f is the difference between the force the library solved with and the
oracle's.  e per form:
  * FP64: the product is two FP64 contractions, sums over the samples (n) and
    over the N + 1 augmented sites; the forward error of such sums is at most
    (n + N + 1) u with u = 2^-53, about 3e-14 for n = 2048 and N = 256, so
    e = 1e-13 covers it with the CG recurrence's own accumulation;
  * FP32 Jacobian / two-term BF16 forms: each entry or operand carries about
    2^-17 relative error and FP32 accumulation adds (sum length) 2^-24; e = 3e-5.
|S + eps I|_2 is estimated by power iteration on the oracle's product."""
import numpy as np
import pytest

import synth
from oracle import core

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible HIP device")
    return torch


def _state(w, **kw):
    from paper_2112_10526_amd.nqs import VMCState
    print(f"[case] {w.name} {kw}", flush=True)
    return VMCState.from_workload(w, **kw)


def _spectral_norm(O, shift, iters=15, seed=0):
    v = np.random.default_rng(seed).normal(size=O.shape[1])
    for _ in range(iters):
        v = core.qgt_matvec(O, v, shift)
        v /= np.linalg.norm(v)
    return np.linalg.norm(core.qgt_matvec(O, v, shift))


def _check(name, O, f, g, d, shift, tol, eps, gnorm):
    res = np.linalg.norm(core.qgt_matvec(O, d, shift) - f)
    bound = 2 * tol * np.linalg.norm(f) + eps * gnorm * np.linalg.norm(d) + np.linalg.norm(g - f)
    print(f"{name}: residual {res:.3e} bound {bound:.3e} |f| {np.linalg.norm(f):.3e} "
          f"|S| {gnorm:.3e} |d| {np.linalg.norm(d):.3e} |g-f| {np.linalg.norm(g - f):.3e}",
          flush=True)
    assert res <= bound, name
    assert bound < 0.1 * np.linalg.norm(f), name  # informative: far below |f|


@pytest.mark.timeout(900)
def test_dense_qgt_full_size_against_oracle():
    """N = 64 Heisenberg chain, alpha = 8 (33,344 parameters), the full 16,384-sample
    batch: the dense Jacobian QGT directions (FP32 Gram on the FP32 matrix cores;
    BF16-split Gram) and the on-the-fly directions of both forms against the
    oracle's product, and the two representations against each other."""
    torch = _torch()
    w = synth.WORKLOADS["heis1d_n64"]
    s = synth.sz0_configs(w.n_samples, w.n_sites, 12)
    tol, shift = 1e-6, 0.01
    dirs = {}
    for precision in ("fp32", "bf16"):
        for qgt in ("onthefly", "jacobian_dense"):
            st = _state(w, precision=precision, qgt=qgt)
            st.load_samples(torch.from_numpy(s))
            _, g = st.expect_and_grad()
            d, info = st.sr_update(qgt=qgt, diag_shift=shift, lr=0.0, tol=tol, maxiter=3000)
            assert info.converged, (precision, qgt, info)
            dirs[(precision, qgt)] = (d.cpu().numpy(), g.cpu().numpy())
            st.close()
            del st
            torch.cuda.empty_cache()
        a, b = dirs[(precision, "onthefly")][0], dirs[(precision, "jacobian_dense")][0]
        assert np.abs(a - b).max() <= 2e-3 * np.abs(a).max(), precision
    rbm = core.Rbm(w.n_sites, w.n_hidden, w.params())
    ham = core.Hamiltonian.heisenberg(w.n_sites, w.bonds(), w.J, w.sublattice())
    print("oracle: local energies, Jacobian, force, |S|", flush=True)
    E = core.local_energy(rbm, ham, s)
    O = core.jacobian(rbm, s)  # 16,384 x 33,344 FP64 (4.4 GB)
    f = core.force(O, E)
    gnorm = _spectral_norm(O, shift)
    for (precision, qgt), (d, g) in dirs.items():
        assert np.abs(g - f).max() <= 2e-4 * np.abs(f).max(), (precision, qgt)
        _check(f"{precision} {qgt}", O, f, g, d, shift, tol, 3e-5, gnorm)


@pytest.mark.timeout(900)
def test_precision_form_shape_sr_direction():
    """16x16 Heisenberg, alpha = 4 (1,024 hidden units, 263,424 parameters), on a
    batch of 2,048 samples drawn by the library's own exchange sampler after
    thermalisation; FP64 path and BF16 form solve on that identical batch."""
    torch = _torch()
    w = synth.WORKLOADS["heis2d_l16"].replace(n_chains=2048)
    tol, shift = 1e-6, 0.01
    st = _state(w, precision="fp64")
    st.thermalize(4)
    smp, _, _ = st.sample()
    s = smp.reshape(-1, w.n_sites).cpu().numpy()
    out = {}
    for precision in ("fp64", "bf16"):
        if precision != "fp64":
            st = _state(w, precision=precision)
        st.load_samples(torch.from_numpy(s))
        _, g = st.expect_and_grad()
        d, info = st.sr_update(diag_shift=shift, lr=0.0, tol=tol, maxiter=4000)
        assert info.converged, (precision, info)
        out[precision] = (d.cpu().numpy(), g.cpu().numpy(), info.iterations)
        st.close()
        del st
        torch.cuda.empty_cache()
    rbm = core.Rbm(w.n_sites, w.n_hidden, w.params())
    ham = core.Hamiltonian.heisenberg(w.n_sites, w.bonds(), w.J, w.sublattice())
    print("oracle: local energies", flush=True)
    E = core.local_energy(rbm, ham, s)
    print("oracle: Jacobian, force, |S|", flush=True)
    O = core.jacobian(rbm, s)  # 2,048 x 263,424 FP64 (4.3 GB)
    f = core.force(O, E)
    gnorm = _spectral_norm(O, shift)
    d, g, _ = out["fp64"]
    assert np.abs(g - f).max() <= 1e-10 * np.abs(f).max()
    _check("fp64", O, f, g, d, shift, tol, 1e-13, gnorm)
    d, g, _ = out["bf16"]
    assert np.abs(g - f).max() <= 2e-4 * np.abs(f).max()
    _check("bf16", O, f, g, d, shift, tol, 3e-5, gnorm)


@pytest.mark.timeout(600)
def test_onthefly_wide_site_tiles_fp64():
    """A 150-site TFIM chain, alpha = 2 (ten 16-site tiles, nineteen 16-unit hidden
    tiles): the contraction-2 blocks of the FP64 path then hold 1,024 threads with
    one site tile per active wave, and the sample ranges split 256 samples over
    13 blocks per hidden tile.  Force and SR direction against the oracle's
    Jacobian on the same random batch (same property as above, FP64 e)."""
    torch = _torch()
    w = synth.WORKLOADS["tfim1d_n10"].replace(L=150, alpha=2, sweep_size=150, n_chains=64,
                                              samples_per_chain=4, sigma=0.05)
    tol, shift = 1e-9, 0.01
    st = _state(w, precision="fp64")
    s = synth.random_configs(w.n_samples, w.n_sites, 21)
    st.load_samples(torch.from_numpy(s).cuda())
    _, g = st.expect_and_grad()
    d, info = st.sr_update(diag_shift=shift, lr=0.0, tol=tol, maxiter=4000)
    assert info.converged, info
    rbm = core.Rbm(w.n_sites, w.n_hidden, w.params())
    ham = core.Hamiltonian.tfim(w.n_sites, w.bonds(), w.J, w.h)
    O = core.jacobian(rbm, s)
    f = core.force(O, core.local_energy(rbm, ham, s))
    g = g.cpu().numpy()
    assert np.abs(g - f).max() <= 1e-10 * np.abs(f).max()
    _check("fp64 wide", O, f, g, d.cpu().numpy(), shift, tol, 1e-13, _spectral_norm(O, shift))
