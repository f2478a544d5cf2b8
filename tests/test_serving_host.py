"""Host logic of the continuous-batching server (no GPU): admission by HBM
footprint in arrival order, slot limits, freeing on completion, rejection of
runs that can never fit; in both serving modes (lock-step ticks, and
asynchronous steps where runs of different step lengths finish out of order)."""
import types

import pytest

from paper_2112_10526_amd.serving import Request, Server


class FakeState:
    live = 0
    peak = 0

    def __init__(self, req, footprint):
        self.req = req
        self.workspace_bytes = footprint
        self.n_samples = req.n_samples
        self.bound = False

    def bind(self):
        self.bound = True
        FakeState.live += self.workspace_bytes
        FakeState.peak = max(FakeState.peak, FakeState.live)

    def thermalize(self, n):
        assert self.bound

    def get_params(self):
        return None

    def close(self):
        if self.bound:
            FakeState.live -= self.workspace_bytes
        self.bound = False


def fake_step(states, cfgs):
    out = []
    for s in states:
        assert s.bound
        out.append(types.SimpleNamespace(energy=dict(mean=-float(s.req.id)),
                                         sr=types.SimpleNamespace(iterations=3)))
    return out


def fake_begin(state, cfg):
    assert state.bound and not getattr(state, "inflight", False)
    state.inflight = True
    state.left = 1 + state.req.id % 3  # polls until this step ends (runs differ)


def fake_poll(states, wait):
    assert any(getattr(s, "inflight", False) for s in states)
    out = {}
    while not out:
        for k, s in enumerate(states):
            if getattr(s, "inflight", False):
                s.left -= 1
                if s.left == 0:
                    s.inflight = False
                    out[k] = types.SimpleNamespace(energy=dict(mean=-float(s.req.id)),
                                                   sr=types.SimpleNamespace(iterations=3))
        if not wait:
            break
    return out


def make_server(budget, slots, sizes, mode="tick"):
    FakeState.live = FakeState.peak = 0
    return Server(budget, max_slots=slots, streams=[None, None],
                  state_factory=lambda req, stream: FakeState(req, sizes[req.id]),
                  step_fn=fake_step, begin_fn=fake_begin, poll_fn=fake_poll, mode=mode)


@pytest.mark.parametrize("mode", ["tick", "async"])
def test_admission_respects_budget_and_order(mode):
    reqs = [Request(k, 0.0, 4, 1.0, 1, 1024, n_steps=2 + k % 3) for k in range(12)]
    sizes = {k: 100 + 10 * k for k in range(12)}
    srv = make_server(budget=400, slots=8, sizes=sizes, mode=mode)
    out = srv.serve(reqs, realtime=False)
    assert FakeState.peak <= 400
    assert FakeState.live == 0
    res = out["results"]
    assert all(len(r.energies) == reqs[r.id].n_steps for r in res.values())
    adm = [res[k].admitted for k in range(12)]
    assert adm == sorted(adm)  # arrival order is kept
    assert out["sr_steps"] == sum(r.n_steps for r in reqs)


@pytest.mark.parametrize("mode", ["tick", "async"])
def test_slot_limit_and_rejection(mode):
    reqs = [Request(k, 0.0, 4, 1.0, 1, 1024, n_steps=3) for k in range(6)]
    sizes = {0: 10, 1: 10, 2: 10_000, 3: 10, 4: 10, 5: 10}
    srv = make_server(budget=1000, slots=2, sizes=sizes, mode=mode)
    out = srv.serve(reqs, realtime=False)
    res = out["results"]
    assert res[2].error is not None and not res[2].energies
    for k in (0, 1, 3, 4, 5):
        assert len(res[k].energies) == 3
    # never more than two resident runs: each tick steps at most two runs
    assert out["ticks"] >= 3 * 5 / 2
    assert out["mean_resident"] <= 2


def test_residency_and_latency_figures():
    # three runs present at the start, two slots: ticks advance 2, 2, 1 runs
    reqs = [Request(k, 0.0, 4, 1.0, 1, 1024, n_steps=2) for k in range(3)]
    srv = make_server(budget=1000, slots=2, sizes={k: 10 for k in range(3)}, mode="tick")
    t = iter(range(10_000))
    calls = []
    out = srv.serve(reqs, clock=lambda: float(next(t)), realtime=False,
                    progress=lambda *a: calls.append(a))
    assert out["sr_steps"] == 6
    assert len(calls) == out["ticks"] and calls[-1] == (3, 3, 6)
    assert out["mean_resident"] == pytest.approx(6 / out["ticks"])
    assert out["queue_delay_ms_p50"] >= 0 and out["queue_delay_ms_p99"] >= out["queue_delay_ms_p50"]
    assert out["run_latency_ms_p99"] >= out["run_latency_ms_p50"] > 0
    assert out["local_energies_per_busy_s"] >= out["local_energies_per_s"] > 0


def test_async_runs_finish_out_of_order_and_refill_slots():
    # run 0 takes one poll per step, run 1 two, run 2 three: with two slots the
    # short run finishes first and run 2 takes its slot while run 1 is mid-step
    reqs = [Request(k, 0.0, 4, 1.0, 1, 1024, n_steps=2) for k in range(3)]
    srv = make_server(budget=1000, slots=2, sizes={k: 10 for k in range(3)}, mode="async")
    t = iter(range(10_000))
    out = srv.serve(reqs, clock=lambda: float(next(t)), realtime=False)
    res = out["results"]
    assert all(len(r.energies) == 2 for r in res.values())
    assert res[0].finished < res[1].finished
    assert res[2].admitted < res[1].finished  # admitted before run 1 was done
    assert FakeState.live == 0 and FakeState.peak <= 20


def test_package_problem_definitions_match_the_test_inputs():
    """The library's own bond lists, sublattices and initial parameters (it does
    not import the test-input module) equal the test inputs' independent ones."""
    import numpy as np

    import synth
    from paper_2112_10526_amd import lattice
    for L in (3, 4, 7, 10, 16):
        np.testing.assert_array_equal(lattice.square_bonds(L), synth.square_bonds(L))
        np.testing.assert_array_equal(lattice.square_sublattice(L), synth.square_sublattice(L))
    for n in (3, 10, 64):
        np.testing.assert_array_equal(lattice.chain_bonds(n), synth.chain_bonds(n))
        np.testing.assert_array_equal(lattice.chain_sublattice(n), synth.chain_sublattice(n))
    np.testing.assert_array_equal(lattice.init_params(100, 200, 1), synth.rbm_params(100, 200, 1))


def test_poisson_stream_is_seeded():
    import numpy as np

    from paper_2112_10526_amd.serving import poisson_stream
    a = poisson_stream(64, seed=7, rate=10.0, n_steps=5)
    b = poisson_stream(64, seed=7, rate=10.0, n_steps=5)
    assert [dataclasses_tuple(r) for r in a] == [dataclasses_tuple(r) for r in b]
    t = np.array([r.arrival for r in a])
    assert np.all(np.diff(t) > 0)
    assert all(4 <= r.L <= 20 and 0.5 <= r.h <= 4.0 and r.alpha in (1, 2, 4) for r in a)
    # mean inter-arrival time 1 / rate within 5 standard errors
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert abs(gaps.mean() - 0.1) < 5 * 0.1 / np.sqrt(gaps.size)


def dataclasses_tuple(r):
    import dataclasses
    return dataclasses.astuple(r)
