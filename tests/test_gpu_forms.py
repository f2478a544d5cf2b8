"""GPU tests of the three additional forms and of the headline workload at full
size: differentiation (autograd function over the hand-written vJp kernel,
dense Jacobian QGT at the N=64 chain size), serving (each run's result is the
same alone and in the mix), and the 10x10 TFIM step in the benchmark's launch
configuration checked against the oracle on sampled chains and by properties."""
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


# ----------------------------------------------------------------------------
# differentiation form
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 3e-5)])
def test_autograd_log_psi_matches_oracle(precision, tol):
    torch = _torch()
    from paper_2112_10526_amd.autograd import log_psi
    w = synth.WORKLOADS["heis1d_n64"].replace(sigma=0.05)
    st = _state(w, precision=precision, n_chains=64)
    s = torch.from_numpy(synth.sz0_configs(2048, w.n_sites, 9)).cuda()
    p = torch.tensor(w.params(), device="cuda", requires_grad=True)
    wts = torch.from_numpy(np.random.default_rng(1).normal(size=2048)).cuda()
    y = log_psi(p, s, st)
    (y.double() * wts).sum().backward()
    rbm = core.Rbm(w.n_sites, w.n_hidden, w.params())
    ref = core.jacobian(rbm, s.cpu().numpy()).T @ wts.cpu().numpy()
    g = p.grad.cpu().numpy()
    assert np.abs(g - ref).max() <= tol * np.abs(ref).max()
    yo = core.log_psi(rbm, s.cpu().numpy())
    assert np.abs(y.detach().double().cpu().numpy() - yo).max() <= (1e-12 if precision == "fp64" else 2e-5) * np.abs(yo).max()


def test_autograd_finite_differences_fp64():
    torch = _torch()
    from paper_2112_10526_amd.autograd import log_psi
    w = synth.WORKLOADS["heis1d_n64"].replace(sigma=0.1, L=16, alpha=2)
    st = _state(w, precision="fp64", n_chains=16)
    s = torch.from_numpy(synth.sz0_configs(64, w.n_sites, 2)).cuda()
    p0 = torch.tensor(w.params(), device="cuda")
    p = p0.clone().requires_grad_(True)
    log_psi(p, s, st).sum().backward()
    g = p.grad.cpu().numpy()
    rng = np.random.default_rng(3)
    h = 1e-5
    for k in rng.choice(p0.numel(), 12, replace=False):
        e = torch.zeros_like(p0)
        e[k] = h
        fp = log_psi(p0 + e, s, st).sum().item()
        fm = log_psi(p0 - e, s, st).sum().item()
        assert abs((fp - fm) / (2 * h) - g[k]) <= 1e-7 * max(1.0, abs(g[k]))


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_dense_qgt_full_size(precision):
    """N = 64 chain, alpha = 8 (33,344 parameters), 16,384 samples: dense
    Jacobian (2.2 GB) + MFMA Gram (4.4 GB; BF16 split in the BF16 form) + CG
    against the on-the-fly solve of the same form."""
    torch = _torch()
    w = synth.WORKLOADS["heis1d_n64"]
    s = torch.from_numpy(synth.sz0_configs(w.n_samples, w.n_sites, 12))
    out = {}
    for qgt in ("onthefly", "jacobian_dense"):
        st = _state(w, precision=precision, qgt=qgt)
        st.load_samples(s)
        st.expect_and_grad()
        d, info = st.sr_update(qgt=qgt, diag_shift=0.01, lr=0.0, tol=1e-6, maxiter=3000)
        assert info.converged, (qgt, info)
        out[qgt] = d.cpu().numpy()
        st.close()
        del st
        torch.cuda.empty_cache()
    a, b = out["onthefly"], out["jacobian_dense"]
    assert np.abs(a - b).max() <= 2e-3 * np.abs(a).max()


# ----------------------------------------------------------------------------
# serving form
# ----------------------------------------------------------------------------
def _serve(reqs, budget, slots=16, precision="bf16", mode="async"):
    from paper_2112_10526_amd.serving import Server
    srv = Server(budget, max_slots=slots, n_streams=4, precision=precision,
                 thermalize_segments=5, keep_params=True, mode=mode)
    return srv.serve(reqs, realtime=False)


# alone: one run at a time in lock-step mode; mixes: all four together, in
# both modes, and with a budget that fits one run at a time
@pytest.mark.parametrize("precision", ["bf16", "fp64"])
def test_serving_result_same_alone_and_in_mix(precision):
    _torch()
    from paper_2112_10526_amd.serving import Request
    reqs = [Request(0, 0.0, 4, 0.8, 1, 1024, 4, 11, 21), Request(1, 0.0, 6, 3.0, 2, 2048, 3, 12, 22),
            Request(2, 0.0, 5, 1.7, 4, 1024, 5, 13, 23), Request(3, 0.0, 7, 2.5, 1, 4096, 2, 14, 24)]
    alone = {}
    for r in reqs:
        out = _serve([r], 1 << 34, precision=precision, mode="tick")
        alone[r.id] = out["results"][r.id]
    mixes = [_serve(reqs, 1 << 34, precision=precision, mode=m)["results"]
             for m in ("tick", "async")]
    tight = _serve(reqs, max(x.footprint for x in alone.values()) + 1, precision=precision)
    for r in reqs:
        a = alone[r.id]
        for other in [m[r.id] for m in mixes] + [tight["results"][r.id]]:
            assert other.energies == a.energies, r.id
            np.testing.assert_array_equal(other.params, a.params)
    assert tight["peak_hbm_bytes"] <= max(x.footprint for x in alone.values()) + 1


def _batch_run(reqs, precisions, steps, grouping):
    """Every request as its own state (4 streams), `steps` batched SR steps;
    per run: the step energies, CG iteration counts and final parameters."""
    torch = _torch()
    from paper_2112_10526_amd.nqs import VMCState, batch_step
    streams = [torch.cuda.Stream() for _ in range(4)]
    sts = []
    for k, (r, prec) in enumerate(zip(reqs, precisions)):
        st = VMCState.from_workload(r.workload(prec), stream=streams[k % 4], allocate=False)
        st.bind()
        st.thermalize(3)
        st.set_cg_grouping(grouping)
        sts.append(st)
    cfg = dict(diag_shift=0.01, lr=0.01, tol=1e-6)
    out = [([], []) for _ in reqs]
    for _ in range(steps):
        for k, rep in enumerate(batch_step(sts, [cfg] * len(sts))):
            out[k][0].append(rep.energy["mean"])
            out[k][1].append(rep.sr.iterations)
    res = [(e, it, st.get_params()) for (e, it), st in zip(out, sts)]
    for st in sts:
        st.close()
    return res


# grouped CG launches against each run's own launches: runs of five different
# contraction-1 block sizes, with an FP64 run and a run too large to group
# (10x10, alpha 2, 16,384 samples) among them, and 34 BF16 runs (two groups: 32
# and 2)
@pytest.mark.parametrize("case", ["mixed_shapes", "two_groups"])
def test_grouped_cg_same_as_own_launches(case):
    from paper_2112_10526_amd.serving import Request
    if case == "mixed_shapes":
        shapes = [(4, 1, 1024), (6, 2, 2048), (5, 4, 1024), (7, 1, 4096), (8, 4, 2048),
                  (6, 2, 1024), (4, 4, 2048), (10, 2, 16384)]
        precs = ["bf16", "bf16", "bf16", "bf16", "bf16", "fp64", "fp32", "bf16"]
        steps = 3
    else:
        shapes = [(4 + k % 3, 1 + k % 2, 1024) for k in range(34)]
        precs = ["bf16"] * 34
        steps = 2
    reqs = [Request(k, 0.0, L, 0.5 + 0.25 * k, a, ns, steps, 100 + k, 200 + k)
            for k, (L, a, ns) in enumerate(shapes)]
    print(f"[case] grouped CG {case}: {len(reqs)} runs", flush=True)
    own = _batch_run(reqs, precs, steps, grouping=False)
    grp = _batch_run(reqs, precs, steps, grouping=True)
    iters = set()
    for k, ((e0, i0, p0), (e1, i1, p1)) in enumerate(zip(own, grp)):
        assert e1 == e0, k
        assert i1 == i0, k
        np.testing.assert_array_equal(p1, p0)
        iters.update(i0)
    assert len(iters) > 1  # the runs stop at different iterations


@pytest.mark.parametrize("mode", ["tick", "async"])
def test_serving_poisson_stream_smoke(mode):
    _torch()
    from paper_2112_10526_amd.serving import requests_from_stream
    reqs = requests_from_stream(8, seed=5, rate=200.0, n_steps=3, L_range=(4, 8),
                                samples=(1024, 2048))
    out = _serve(reqs, 2 << 30, mode=mode)
    assert out["sr_steps"] == 24
    assert out["p99_step_ms"] >= out["p50_step_ms"] > 0
    for r in out["results"].values():
        assert np.all(np.isfinite(r.energies)) and len(r.energies) == 3


# ----------------------------------------------------------------------------
# headline workload, full size, benchmark launch configuration
# ----------------------------------------------------------------------------
def test_tfim2d_full_size_step_fp64():
    torch = _torch()
    w = synth.WORKLOADS["tfim2d_l10"]
    st = _state(w, precision="fp64")
    ch0 = st.get_chains()
    smp, acc, a = st.sample(log_accepts=True)
    rbm = core.Rbm(w.n_sites, w.n_hidden, w.params())
    ham = core.Hamiltonian.tfim(w.n_sites, w.bonds(), w.J, w.h)
    # sampled chains, bit-exact (chain ids 0..31 and 4064..4095)
    for c0 in (0, 4064):
        ref = core.sample(rbm, ch0[c0:c0 + 32], w.samples_per_chain, w.sweep_size, w.chain_seed,
                          0, chain_offset=c0, mode="cached", log_accepts=True)
        assert ref.margins.min() > 1e-12
        np.testing.assert_array_equal(acc[c0:c0 + 32].cpu().numpy(), ref.accepts)
        np.testing.assert_array_equal(smp[c0:c0 + 32].cpu().numpy(), ref.samples)
    flat = smp.reshape(-1, w.n_sites).cpu().numpy()
    # energies and gradient of the whole batch
    stats, g = st.expect_and_grad()
    E = core.local_energy(rbm, ham, flat)
    assert abs(stats["mean"] - E.mean()) <= 1e-10 * abs(E.mean())
    idx = np.random.default_rng(0).choice(flat.shape[0], 256, replace=False)
    e_gpu = st.local_energy(torch.from_numpy(flat[idx])).cpu().numpy()
    assert np.abs(e_gpu - E[idx]).max() <= 1e-10 * np.abs(E[idx]).max()
    # the SR direction solves the oracle's system to the CG tolerance
    d, info = st.sr_update(diag_shift=0.01, lr=0.0, tol=1e-6)
    assert info.converged
    O = core.jacobian(rbm, flat)
    f = core.force(O, E)
    assert np.abs(g.cpu().numpy() - f).max() <= 1e-10 * np.abs(f).max()
    dd = d.cpu().numpy()
    res = core.qgt_matvec(O, dd, 0.01) - f
    assert np.linalg.norm(res) <= 2e-6 * np.linalg.norm(f)


@pytest.mark.parametrize("precision", ["bf16", "fp32"])
def test_tfim2d_full_size_reduced_precision_energy(precision):
    """The BF16/FP32 forms on the identical full batch: energies within 1e-4."""
    torch = _torch()
    w = synth.WORKLOADS["tfim2d_l10"].replace(sigma=0.05)
    s = synth.random_configs(w.n_samples, w.n_sites, 99)
    st = _state(w, precision=precision)
    e = st.local_energy(torch.from_numpy(s)).cpu().numpy()
    rbm = core.Rbm(w.n_sites, w.n_hidden, w.params())
    ham = core.Hamiltonian.tfim(w.n_sites, w.bonds(), w.J, w.h)
    idx = np.random.default_rng(1).choice(w.n_samples, 512, replace=False)
    ref = core.local_energy(rbm, ham, s[idx])
    assert (np.abs(e[idx] - ref) / np.abs(ref)).max() <= 1e-4


def test_tfim2d_full_size_sr_direction_bf16():
    """BF16 form at full size, in the benchmark's configuration: on the batch its own
    sampler drew, the force is within 2e-4 of the oracle's (FP64) and the CG direction
    solves the oracle's SR system up to the CG tolerance, the rounding of the form's
    operator (eps |G|_2 |d|, eps = 3e-5: two-term BF16 operands, FP32 accumulation) and
    the force difference: |G d - f| <= 2 tol |f| + eps |G|_2 |d| + |g - f|."""
    w = synth.WORKLOADS["tfim2d_l10"]
    st = _state(w, precision="bf16")
    smp, _, _ = st.sample()
    flat = smp.reshape(-1, w.n_sites).cpu().numpy()
    _, g = st.expect_and_grad()
    tol = 1e-6
    d, info = st.sr_update(diag_shift=w.diag_shift, lr=0.0, tol=tol)
    assert info.converged, info
    rbm = core.Rbm(w.n_sites, w.n_hidden, w.params())
    ham = core.Hamiltonian.tfim(w.n_sites, w.bonds(), w.J, w.h)
    E = core.local_energy(rbm, ham, flat)
    O = core.jacobian(rbm, flat)
    f = core.force(O, E)
    g = g.cpu().numpy()
    assert np.abs(g - f).max() <= 2e-4 * np.abs(f).max()
    dd = d.cpu().numpy()
    v = np.random.default_rng(0).normal(size=dd.size)
    for _ in range(20):  # |G|_2 by power iteration on the oracle's product
        v = core.qgt_matvec(O, v, w.diag_shift)
        v /= np.linalg.norm(v)
    gnorm = np.linalg.norm(core.qgt_matvec(O, v, w.diag_shift))
    res = np.linalg.norm(core.qgt_matvec(O, dd, w.diag_shift) - f)
    bound = 2 * tol * np.linalg.norm(f) + 3e-5 * gnorm * np.linalg.norm(dd) + np.linalg.norm(g - f)
    print(f"residual {res:.3e} bound {bound:.3e} |f| {np.linalg.norm(f):.3e} |G| {gnorm:.3e} "
          f"|d| {np.linalg.norm(dd):.3e} |g - f| {np.linalg.norm(g - f):.3e}")
    assert res <= bound
    assert bound < 0.05 * np.linalg.norm(f)  # informative: far below |f|


def test_async_step_same_as_vmc_step():
    """nqs_step_begin / nqs_step_poll give the same step as nqs_vmc_step (twin
    states, same seeds), and a second begin while a step is in flight, or a
    fused step on that context, is refused with NQS_ESTATE."""
    torch = _torch()
    from paper_2112_10526_amd import _lib
    from paper_2112_10526_amd.nqs import NqsError, VMCState, step_begin, step_poll
    w = synth.WORKLOADS["tfim2d_l10"].replace(n_chains=256, sigma=0.05)
    a = VMCState.from_workload(w, precision="bf16")
    b = VMCState.from_workload(w, precision="bf16")
    cfg = dict(diag_shift=w.diag_shift, lr=w.lr, tol=w.cg_tol)
    for _ in range(3):
        ra = a.vmc_step(**{"diag_shift": w.diag_shift, "lr": w.lr, "tol": w.cg_tol})
        step_begin(b, cfg)
        with pytest.raises(NqsError) as e:
            step_begin(b, cfg)
        assert e.value.status == _lib.NQS_ESTATE
        with pytest.raises(NqsError):
            b.vmc_step(diag_shift=w.diag_shift, lr=w.lr, tol=w.cg_tol)
        done = {}
        while not done:
            done = step_poll([b], wait=True)
        rb = done[0]
        assert rb.energy["mean"] == ra.energy["mean"]
        assert rb.sr.iterations == ra.sr.iterations
        np.testing.assert_array_equal(b.get_params(), a.get_params())
    assert step_poll([a, b], wait=True) == {}  # nothing in flight
    a.close()
    b.close()


def test_step_log_lines(tmp_path):
    """The per-step JSON-lines log: one line per SR step with the step's energy
    statistics, acceptance and CG figures, and per-stage kernel times on request."""
    import json
    _torch()
    w = synth.WORKLOADS["tfim2d_l10"].replace(n_chains=256, sigma=0.05)
    st = _state(w, precision="bf16")
    path = tmp_path / "steps.jsonl"
    st.open_step_log(str(path), stage_times=True)
    reps = [st.vmc_step(diag_shift=w.diag_shift, lr=w.lr, tol=w.cg_tol) for _ in range(3)]
    st.close_step_log()
    st.vmc_step(diag_shift=w.diag_shift, lr=w.lr, tol=w.cg_tol)  # not logged
    st.close()
    lines = [json.loads(x) for x in path.read_text().splitlines()]
    assert [x["step"] for x in lines] == [1, 2, 3]
    for x, r in zip(lines, reps):
        assert x["energy"] == r.energy["mean"] and x["cg_iters"] == r.sr.iterations
        assert x["acceptance"] == r.energy["acceptance"] and x["wall_ms"] > 0
        assert {"sample", "eloc", "qgt_w", "outer"} <= set(x["stage_ms"])
