"""Host logic of the continuous-batching server (no GPU): admission by HBM
footprint in arrival order, slot limits, freeing on completion, rejection of
runs that can never fit."""
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


def make_server(budget, slots, sizes):
    FakeState.live = FakeState.peak = 0
    return Server(budget, max_slots=slots, streams=[None, None],
                  state_factory=lambda req, stream: FakeState(req, sizes[req.id]),
                  step_fn=fake_step)


def test_admission_respects_budget_and_order():
    reqs = [Request(k, 0.0, 4, 1.0, 1, 1024, n_steps=2 + k % 3) for k in range(12)]
    sizes = {k: 100 + 10 * k for k in range(12)}
    srv = make_server(budget=400, slots=8, sizes=sizes)
    out = srv.serve(reqs, realtime=False)
    assert FakeState.peak <= 400
    assert FakeState.live == 0
    res = out["results"]
    assert all(len(r.energies) == reqs[r.id].n_steps for r in res.values())
    adm = [res[k].admitted for k in range(12)]
    assert adm == sorted(adm)  # arrival order is kept
    assert out["sr_steps"] == sum(r.n_steps for r in reqs)


def test_slot_limit_and_rejection():
    reqs = [Request(k, 0.0, 4, 1.0, 1, 1024, n_steps=3) for k in range(6)]
    sizes = {0: 10, 1: 10, 2: 10_000, 3: 10, 4: 10, 5: 10}
    srv = make_server(budget=1000, slots=2, sizes=sizes)
    out = srv.serve(reqs, realtime=False)
    res = out["results"]
    assert res[2].error is not None and not res[2].energies
    for k in (0, 1, 3, 4, 5):
        assert len(res[k].energies) == 3
    # never more than two resident runs: each tick steps at most two runs
    assert out["ticks"] >= 3 * 5 / 2


def test_residency_and_latency_figures():
    # three runs present at the start, two slots: ticks advance 2, 2, 1 runs
    reqs = [Request(k, 0.0, 4, 1.0, 1, 1024, n_steps=2) for k in range(3)]
    srv = make_server(budget=1000, slots=2, sizes={k: 10 for k in range(3)})
    t = iter(range(10_000))
    out = srv.serve(reqs, clock=lambda: float(next(t)), realtime=False)
    assert out["sr_steps"] == 6
    assert out["mean_resident"] == pytest.approx(6 / out["ticks"])
    assert out["queue_delay_ms_p50"] >= 0 and out["queue_delay_ms_p99"] >= out["queue_delay_ms_p50"]
    assert out["run_latency_ms_p99"] >= out["run_latency_ms_p50"] > 0
    assert out["local_energies_per_busy_s"] >= out["local_energies_per_s"] > 0
