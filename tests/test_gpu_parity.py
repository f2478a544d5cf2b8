"""GPU-vs-oracle parity through the C ABI (libnqs) on seeded synthetic inputs.

Bars (derived in the design notes):
  * chain starts, configurations and Metropolis accept/reject sequences:
    bit-exact with the oracle in FP64 (the smallest |u - ratio^2| of the
    oracle is logged and must exceed 1e-12 so no decision is ambiguous);
  * FP64 local energies, log-amplitudes and force: |gpu - oracle| <=
    1e-10 * max(|oracle|, 1) (force: relative to its largest component);
  * FP32 and BF16 forms: local energies within 1e-4 relative;
  * SR directions: against the oracle's Cholesky solve of the same system.
"""
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


def make_state(w, precision=None, n_chains=None, params=None, qgt="onthefly", **kw):
    _torch()
    from paper_2112_10526_amd.nqs import VMCState
    w2 = w.replace(**kw) if kw else w
    print(f"[case] {w2.name} prec={precision or w2.precision} chains={n_chains or w2.n_chains}",
          flush=True)
    return VMCState.from_workload(w2, precision=precision, n_chains=n_chains, params=params,
                                  qgt=qgt), w2


def oracle_model(w, params):
    rbm = core.Rbm(w.n_sites, w.n_hidden, params)
    if w.model == "tfim":
        ham = core.Hamiltonian.tfim(w.n_sites, w.bonds(), w.J, w.h)
    else:
        ham = core.Hamiltonian.heisenberg(w.n_sites, w.bonds(), w.J, w.sublattice())
    return rbm, ham


def rel_close(a, b, tol):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    scale = np.maximum(np.abs(b), 1.0)
    err = np.abs(a - b) / scale
    assert err.max() <= tol, f"max rel err {err.max():.3e} > {tol:.1e} at {int(err.argmax())}"


TFIM1D = synth.WORKLOADS["tfim1d_n10"]
TFIM2D = synth.WORKLOADS["tfim2d_l10"]
HEIS2D = synth.WORKLOADS["heis2d_l16"]
HEIS1D = synth.WORKLOADS["heis1d_n64"]


# ----------------------------------------------------------------------------
# chains and sampler
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("sz0", [False, True])
def test_chain_starts_bit_exact(sz0):
    w = TFIM2D.replace(total_sz_zero=sz0)
    st, w = make_state(w, n_chains=300)
    got = st.get_chains()
    ref = core.init_chains(w.n_sites, 300, w.chain_seed, 0, sz0)
    np.testing.assert_array_equal(got, ref)


# (an even chain count pairs two chains per wave; an odd one runs one per wave)
@pytest.mark.parametrize("wname,chains,sigma", [("tfim1d_n10", 16, 0.01), ("tfim1d_n10", 16, 0.3),
                                                ("tfim2d_l10", 128, 0.01), ("tfim2d_l10", 64, 0.1),
                                                ("tfim2d_l10", 63, 0.1), ("tfim1d_n10", 15, 0.3)])
def test_local_sampler_bit_exact_fp64(wname, chains, sigma):
    w = synth.WORKLOADS[wname].replace(sigma=sigma)
    st, w = make_state(w, precision="fp64", n_chains=chains)
    ch0 = st.get_chains()
    smp, acc, a = st.sample(log_accepts=True)
    rbm, _ = oracle_model(w, w.params())
    ref = core.sample(rbm, ch0, w.samples_per_chain, w.sweep_size, w.chain_seed, 0,
                      mode="cached", log_accepts=True)
    assert ref.margins.min() > 1e-12
    np.testing.assert_array_equal(acc.cpu().numpy(), ref.accepts)
    np.testing.assert_array_equal(smp.cpu().numpy(), ref.samples)
    np.testing.assert_array_equal(st.get_chains(), ref.chains)
    assert abs(a - ref.n_accepted.sum() / ref.accepts.size) < 1e-15
    # a second call continues the same streams
    smp2, acc2, _ = st.sample(log_accepts=True)
    ref2 = core.sample(rbm, ref.chains, w.samples_per_chain, w.sweep_size, w.chain_seed,
                       w.samples_per_chain * w.sweep_size, mode="cached", log_accepts=True)
    assert ref2.margins.min() > 1e-12
    np.testing.assert_array_equal(acc2.cpu().numpy(), ref2.accepts)
    np.testing.assert_array_equal(smp2.cpu().numpy(), ref2.samples)


# alpha 4: 1024 hidden units (one chain per wave); alpha 1: 256 (two chains per wave
# with an even chain count, one with an odd count)
@pytest.mark.parametrize("alpha,chains", [(4, 64), (1, 64), (1, 63)])
def test_exchange_sampler_bit_exact_fp64(alpha, chains):
    w = HEIS2D.replace(sigma=0.05, samples_per_chain=2, alpha=alpha)
    st, w = make_state(w, precision="fp64", n_chains=chains)
    ch0 = st.get_chains()
    assert (ch0.astype(int).sum(axis=1) == 0).all()
    smp, acc, _ = st.sample(log_accepts=True)
    rbm, _ = oracle_model(w, w.params())
    ref = core.sample(rbm, ch0, w.samples_per_chain, w.sweep_size, w.chain_seed, 0,
                      rule="exchange", bonds=w.bonds(), mode="cached", log_accepts=True)
    assert ref.margins.min() > 1e-12
    np.testing.assert_array_equal(acc.cpu().numpy(), ref.accepts)
    np.testing.assert_array_equal(smp.cpu().numpy(), ref.samples)


def test_thermalization_and_counter():
    w = TFIM1D.replace(sigma=0.2)
    st, w = make_state(w, precision="fp64")
    ch0 = st.get_chains()
    st.thermalize(7)
    assert st.proposal_count == 7 * w.sweep_size
    rbm, _ = oracle_model(w, w.params())
    ref = core.sample(rbm, ch0, 7, w.sweep_size, w.chain_seed, 0, mode="cached")
    np.testing.assert_array_equal(st.get_chains(), ref.chains)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_reduced_precision_sampler_statistics(precision):
    # FP32/BF16 chains are not bit-exact; their decisions must agree with FP64
    # except near ties, so almost all accept flags coincide on the first segment.
    w = TFIM2D.replace(samples_per_chain=1)
    st64, _ = make_state(w, precision="fp64", n_chains=256)
    st32, _ = make_state(w, precision=precision, n_chains=256)
    _, a64, r64 = st64.sample(log_accepts=True)
    _, a32, r32 = st32.sample(log_accepts=True)
    same = (a64.cpu().numpy() == a32.cpu().numpy()).all(axis=1)
    # until the first differing decision everything is identical
    assert same.mean() > 0.9, same.mean()
    assert abs(r64 - r32) < 0.02


# ----------------------------------------------------------------------------
# local energies and log-amplitudes on identical batches
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("wname", ["tfim1d_n10", "tfim2d_l10", "heis2d_l16", "heis1d_n64"])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-4), ("bf16", 1e-4)])
def test_local_energy_parity(wname, precision, tol):
    torch = _torch()
    w = synth.WORKLOADS[wname].replace(sigma=0.05)
    params = w.params()
    st, w = make_state(w, precision=precision, n_chains=64, params=params)
    n = 333  # ragged: not a multiple of any tile
    if w.total_sz_zero:
        s = synth.sz0_configs(n, w.n_sites, 17)
    else:
        s = synth.random_configs(n, w.n_sites, 17)
    e = st.local_energy(torch.from_numpy(s)).cpu().numpy()
    rbm, ham = oracle_model(w, params)
    ref = core.local_energy(rbm, ham, s)
    rel_close(e, ref, tol)
    # empty batch
    assert st.local_energy(torch.zeros((0, w.n_sites), dtype=torch.int8)).numel() == 0


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 2e-5)])
def test_log_psi_parity(precision, tol):
    torch = _torch()
    w = TFIM2D.replace(sigma=0.1)
    params = w.params()
    st, w = make_state(w, precision=precision, n_chains=64, params=params)
    s = synth.random_configs(200, w.n_sites, 5)
    got = st.log_psi(torch.from_numpy(s)).double().cpu().numpy()
    rbm, _ = oracle_model(w, params)
    rel_close(got, core.log_psi(rbm, s), tol)


# ----------------------------------------------------------------------------
# force and SR on identical batches
# ----------------------------------------------------------------------------
def _batch(w, seed):
    if w.total_sz_zero:
        return synth.sz0_configs(w.n_samples, w.n_sites, seed)
    return synth.random_configs(w.n_samples, w.n_sites, seed)


@pytest.mark.parametrize("wname,chains", [("tfim1d_n10", 16), ("tfim2d_l10", 256),
                                          ("heis1d_n64", 128)])
def test_force_parity_fp64(wname, chains):
    torch = _torch()
    w = synth.WORKLOADS[wname].replace(sigma=0.05, n_chains=chains)
    params = w.params()
    st, w = make_state(w, precision="fp64", params=params)
    s = _batch(w, 23)
    st.load_samples(torch.from_numpy(s))
    stats, g = st.expect_and_grad()
    rbm, ham = oracle_model(w, params)
    E = core.local_energy(rbm, ham, s)
    ref = core.energy_stats(E)
    assert abs(stats["mean"] - ref["mean"]) <= 1e-10 * max(abs(ref["mean"]), 1)
    assert abs(stats["variance"] - ref["variance"]) <= 1e-9 * max(abs(ref["variance"]), 1e-3)
    f = core.force(core.jacobian(rbm, s), E)
    gg = g.cpu().numpy()
    assert np.abs(gg - f).max() <= 1e-10 * np.abs(f).max()


@pytest.mark.parametrize("precision,ftol", [("fp32", 2e-4), ("bf16", 2e-4)])
def test_force_reduced_precision(precision, ftol):
    torch = _torch()
    w = TFIM2D.replace(sigma=0.05, n_chains=256)
    params = w.params()
    st, w = make_state(w, precision=precision, params=params)
    s = _batch(w, 29)
    st.load_samples(torch.from_numpy(s))
    stats, g = st.expect_and_grad()
    rbm, ham = oracle_model(w, params)
    E = core.local_energy(rbm, ham, s)
    assert abs(stats["mean"] - E.mean()) <= 1e-4 * abs(E.mean())
    f = core.force(core.jacobian(rbm, s), E)
    assert np.abs(g.cpu().numpy() - f).max() <= ftol * np.abs(f).max()


@pytest.mark.parametrize("wname,chains", [("tfim1d_n10", 16), ("tfim2d_l10", 128)])
def test_sr_direction_parity_fp64(wname, chains):
    torch = _torch()
    w = synth.WORKLOADS[wname].replace(sigma=0.05, n_chains=chains)
    params = w.params()
    st, w = make_state(w, precision="fp64", params=params)
    s = _batch(w, 31)
    st.load_samples(torch.from_numpy(s))
    st.expect_and_grad()
    delta, info = st.sr_update(diag_shift=0.01, lr=0.0, tol=1e-10, maxiter=5000)
    assert info.converged
    rbm, ham = oracle_model(w, params)
    O = core.jacobian(rbm, s)
    E = core.local_energy(rbm, ham, s)
    f = core.force(O, E)
    ref = core.cholesky_solve(core.qgt_dense(O), f, 0.01)
    d = delta.cpu().numpy()
    assert np.abs(d - ref).max() <= 1e-7 * np.abs(ref).max()
    # the oracle's own CG at the production tolerance agrees to that tolerance
    _, dcg, it, res, conv = core.sr_direction(O, E, 0.01, 1e-6)
    assert np.abs(dcg - ref).max() <= 1e-3 * np.abs(ref).max()
    # parameters untouched at lr = 0
    np.testing.assert_allclose(st.get_params(), params, rtol=0, atol=0)


@pytest.mark.parametrize("precision,eps", [("fp64", 1e-13), ("fp32", 3e-5), ("bf16", 3e-5)])
def test_sr_direction_many_sites(precision, eps):
    """16x16 Heisenberg (N = 256, M = 256, 66,048 parameters; several site and hidden
    tile groups per block) on a ragged batch of 333 samples: the CG direction
    satisfies the oracle's SR system up to the CG tolerance plus the rounding of
    the form's operator, |G d - f| <= 2 tol |f| + eps |G|_2 |d|.  eps, FP64 path:
    the product is two FP64 contractions, sums over the n = 333 samples and the
    N + 1 = 257 augmented sites, whose forward error is at most (n + N + 1) u =
    590 x 2^-53 = 6.6e-14 relative to |G| |d|; eps = 1e-13 covers it.  FP32 and
    BF16 forms (both contractions take their operands as two BF16 terms on MFMA
    with FP32 accumulation, relative error about 2^-16 per Jacobian entry, so
    2 x 2^-16 in G, with margin): eps = 3e-5."""
    torch = _torch()
    w = HEIS2D.replace(sigma=0.05, alpha=1, n_chains=111, samples_per_chain=3)
    params = w.params()
    st, w = make_state(w, precision=precision, params=params)
    s = synth.sz0_configs(333, w.n_sites, 43)
    st.load_samples(torch.from_numpy(s))
    st.expect_and_grad()
    tol = 1e-6
    delta, info = st.sr_update(diag_shift=0.01, lr=0.0, tol=tol, maxiter=4000)
    assert info.converged, info
    rbm, ham = oracle_model(w, params)
    O = core.jacobian(rbm, s)
    E = core.local_energy(rbm, ham, s)
    f = core.force(O, E)
    d = delta.cpu().numpy()
    res = np.linalg.norm(core.qgt_matvec(O, d, 0.01) - f)
    # |G|_2 by power iteration on the oracle's product
    v = np.random.default_rng(0).normal(size=d.size)
    for _ in range(40):
        v = core.qgt_matvec(O, v, 0.01)
        v /= np.linalg.norm(v)
    gnorm = np.linalg.norm(core.qgt_matvec(O, v, 0.01))
    bound = 2 * tol * np.linalg.norm(f) + eps * gnorm * np.linalg.norm(d)
    print(f"residual {res:.3e} bound {bound:.3e} |f| {np.linalg.norm(f):.3e} "
          f"|G| {gnorm:.3e} |d| {np.linalg.norm(d):.3e} iterations {info.iterations}")
    assert res <= bound
    # the bound is informative: far below |f| (a wrong direction misses by ~|f|)
    assert bound < 0.2 * np.linalg.norm(f)


@pytest.mark.parametrize("precision", ["fp64", "bf16"])
def test_cg_graph_replay_matches_stream_launches(precision):
    """Graph-replayed CG batches give bit-identical solves to stream launches,
    on several solves in a row with other work between them (the graphs are
    captured once and replayed)."""
    torch = _torch()
    w = TFIM2D.replace(sigma=0.05, n_chains=256)
    params = w.params()
    out = {}
    for graphs in (True, False):
        st, w2 = make_state(w, precision=precision, params=params)
        st.set_cg_graphs(graphs)
        res = []
        for seed in (51, 52, 53):
            st.load_samples(torch.from_numpy(_batch(w2, seed)))
            st.local_energy(torch.from_numpy(_batch(w2, seed + 10)[:64]))
            st.expect_and_grad()
            d, info = st.sr_update(diag_shift=0.01, lr=0.0, tol=1e-8, maxiter=2000)
            assert info.converged and info.iterations > 20, info
            res.append((d.cpu().numpy().copy(), info.iterations))
        out[graphs] = res
    for (a, ia), (b, ib) in zip(out[True], out[False]):
        assert ia == ib
        np.testing.assert_array_equal(a, b)


def test_sr_update_applies_step():
    torch = _torch()
    w = TFIM1D.replace(sigma=0.05)
    params = w.params()
    st, w = make_state(w, precision="fp64", params=params)
    s = _batch(w, 37)
    st.load_samples(torch.from_numpy(s))
    st.expect_and_grad()
    delta, info = st.sr_update(diag_shift=0.01, lr=0.05, tol=1e-8)
    np.testing.assert_allclose(st.get_params(), params - 0.05 * delta.cpu().numpy(), rtol=0,
                               atol=1e-15)


def test_cg_maxiter_reports_notconv():
    torch = _torch()
    w = TFIM1D.replace(sigma=0.05)
    st, w = make_state(w, precision="fp64")
    st.load_samples(torch.from_numpy(_batch(w, 41)))
    st.expect_and_grad()
    from paper_2112_10526_amd._lib import NqsError
    with pytest.raises(NqsError) as e:
        st.sr_update(tol=1e-12, maxiter=1)
    assert e.value.status == 5
    # allowed explicitly: the step is still applied and reported
    st.load_samples(torch.from_numpy(_batch(w, 41)))
    st.expect_and_grad()
    _, info = st.sr_update(tol=1e-12, maxiter=1, allow_notconv=True)
    assert info.iterations == 1 and not info.converged


# ----------------------------------------------------------------------------
# Jacobian, vJp and dense QGT
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-13), ("fp32", 2e-6)])
@pytest.mark.parametrize("center", [False, True])
def test_jacobian_parity(precision, tol, center):
    torch = _torch()
    w = HEIS1D.replace(sigma=0.05, L=16, alpha=2)
    params = w.params()
    st, w = make_state(w, precision=precision, n_chains=64, params=params)
    s = synth.sz0_configs(150, w.n_sites, 3)
    O = st.jacobian(torch.from_numpy(s), center=center).double().cpu().numpy()
    rbm, _ = oracle_model(w, params)
    ref = core.jacobian(rbm, s)
    if center:
        ref = (ref - ref.mean(axis=0)) / np.sqrt(ref.shape[0])
    assert np.abs(O - ref).max() <= tol


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 2e-5)])
def test_vjp_parity(precision, tol):
    torch = _torch()
    w = HEIS1D.replace(sigma=0.05)
    params = w.params()
    st, w = make_state(w, precision=precision, n_chains=64, params=params)
    s = synth.sz0_configs(500, w.n_sites, 4)
    g = np.random.default_rng(0).normal(size=500)
    got = st.log_psi_vjp(torch.from_numpy(s), torch.from_numpy(g)).double().cpu().numpy()
    rbm, _ = oracle_model(w, params)
    ref = core.jacobian(rbm, s).T @ g
    assert np.abs(got - ref).max() <= tol * np.abs(ref).max()


# (ragged: 39 samples, not a multiple of the centring kernel's 8-row blocks, and
# N = 10 sites, so 4-column groups of the weight block straddle hidden rows)
@pytest.mark.parametrize("shape", [dict(L=16, alpha=2, n_chains=64, samples_per_chain=4),
                                   dict(L=10, alpha=1, n_chains=13, samples_per_chain=3)],
                         ids=["n16", "ragged"])
@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16"])
def test_dense_qgt_matches_onthefly(precision, shape):
    torch = _torch()
    w = HEIS1D.replace(sigma=0.05, **shape)
    params = w.params()
    s = _batch(w, 8)
    out = {}
    for qgt in ("onthefly", "jacobian_dense"):
        st, _ = make_state(w, precision=precision, params=params, qgt=qgt)
        st.load_samples(torch.from_numpy(s))
        st.expect_and_grad()
        d, info = st.sr_update(qgt=qgt, diag_shift=0.01, lr=0.0, tol=1e-9, maxiter=4000)
        assert info.converged, (qgt, info)
        out[qgt] = d.cpu().numpy()
    rbm, ham = oracle_model(w, params)
    O = core.jacobian(rbm, s)
    ref = core.cholesky_solve(core.qgt_dense(O), core.force(O, core.local_energy(rbm, ham, s)), 0.01)
    tol = 1e-7 if precision == "fp64" else 2e-3
    for k, d in out.items():
        assert np.abs(d - ref).max() <= tol * np.abs(ref).max(), k


# ----------------------------------------------------------------------------
# whole VMC steps
# ----------------------------------------------------------------------------
def test_vmc_steps_track_oracle_fp64():
    w = TFIM1D.replace(sigma=0.05)
    st, w = make_state(w, precision="fp64")
    rbm, ham = oracle_model(w, w.params())
    ch = st.get_chains()
    prop = 0
    for step in range(3):
        rep = st.vmc_step(diag_shift=w.diag_shift, lr=0.02, tol=1e-10, maxiter=2000)
        rbm, ch, orep = core.vmc_step(rbm, ham, ch, w.samples_per_chain, w.sweep_size,
                                      w.chain_seed, prop, "local", w.diag_shift, 0.02, 1e-10, 2000)
        prop += w.samples_per_chain * w.sweep_size
        np.testing.assert_array_equal(st.get_chains(), ch)
        assert abs(rep.energy["mean"] - orep.energy["mean"]) <= 1e-10 * abs(orep.energy["mean"])
        assert np.abs(st.get_params() - rbm.params).max() <= 1e-9


def test_vmc_steps_track_oracle_heisenberg_exchange_fp64():
    """Three whole steps of the Heisenberg chain (N = 10, Marshall-rotated, zero
    magnetisation, exchange moves over the bonds): chains bit-exact, energies within
    1e-10 and parameters within 1e-9 of the oracle's steps."""
    w = HEIS1D.replace(L=10, alpha=2, n_chains=32, samples_per_chain=8, sweep_size=10,
                       sigma=0.05)
    st, w = make_state(w, precision="fp64")
    rbm, ham = oracle_model(w, w.params())
    ch = st.get_chains()
    assert (ch.astype(int).sum(axis=1) == 0).all()
    prop = 0
    for step in range(3):
        rep = st.vmc_step(diag_shift=w.diag_shift, lr=0.02, tol=1e-10, maxiter=2000)
        rbm, ch, orep = core.vmc_step(rbm, ham, ch, w.samples_per_chain, w.sweep_size,
                                      w.chain_seed, prop, "exchange", w.diag_shift, 0.02, 1e-10,
                                      2000)
        prop += w.samples_per_chain * w.sweep_size
        np.testing.assert_array_equal(st.get_chains(), ch)
        assert abs(rep.energy["mean"] - orep.energy["mean"]) <= 1e-10 * abs(orep.energy["mean"])
        assert np.abs(st.get_params() - rbm.params).max() <= 1e-9


@pytest.mark.parametrize("precision", ["fp64", "bf16"])
def test_vmc_converges_tfim_chain_gpu(precision):
    """SR from small random parameters reaches the exact ground energy of the
    periodic N = 10 chain (Pfeuty closed form) within 0.3 % in both forms."""
    w = TFIM1D
    st, w = make_state(w, precision=precision)
    st.thermalize(100)
    E = [st.vmc_step(lr=0.05).energy["mean"] for _ in range(150)]
    from oracle import exact
    e0 = exact.tfim_chain_ground_energy(10, 1.0, 1.0)
    assert abs(np.mean(E[-20:]) - e0) < 0.003 * abs(e0)


def test_checkpoint_resume_bit_exact():
    w = TFIM1D.replace(sigma=0.05)
    st, w = make_state(w, precision="fp64")
    st.vmc_step()
    blob = st.get_state()
    a = [st.vmc_step().energy["mean"] for _ in range(3)]
    pa = st.get_params()
    st.set_state(blob)
    b = [st.vmc_step().energy["mean"] for _ in range(3)]
    assert a == b
    np.testing.assert_array_equal(st.get_params(), pa)


def test_invalid_inputs_rejected():
    _torch()
    from paper_2112_10526_amd.nqs import VMCState
    from paper_2112_10526_amd._lib import NqsError
    with pytest.raises(NqsError) as e:
        VMCState(model="tfim", n_sites=4, bonds=[[0, 1], [1, 7]], J=1.0, h=1.0, n_hidden=4,
                 n_chains=4, samples_per_chain=1, sweep_size=4, seed=1)
    assert e.value.status == 1
    w = TFIM1D
    st, w = make_state(w)
    bad = w.params()
    bad[3] = np.nan
    with pytest.raises(NqsError) as e:
        st.set_params(bad)
    assert e.value.status == 4
