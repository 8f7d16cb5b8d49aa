"""Host logic of serving (no GPU): the request stream's shape, workspace
sizing, and the continuous-batching loop driven by a stand-in executor that
records every fused call (admission order, slot and memory limits, joins
between calls, every request stepped exactly its number of steps)."""
import numpy as np
import pytest

from paper_1101_4127_amd import rt, serve
from paper_1101_4127_amd import workloads as W


def test_request_stream_has_the_stated_shape():
    reqs = W.serving_stream(count=512, seed=4)
    t = np.array([r.arrival_s for r in reqs])
    assert np.all(np.diff(t) > 0)
    # Poisson arrivals of mean rate 200/s: gaps pooled over eight streams
    # (4096 exponential gaps: the mean is within 5 % of 1/200 s at > 3 sigma)
    gaps = np.concatenate([np.diff(np.concatenate([[0.0], [q.arrival_s for q in W.serving_stream(count=512, seed=s, sides=(16,))]]))
                           for s in range(4, 12)])
    assert abs(gaps.mean() * 200.0 - 1.0) < 0.05
    assert abs(np.std(gaps) / gaps.mean() - 1.0) < 0.08     # exponential: std = mean
    sides = {r.work.n[0] for r in reqs}
    assert sides == {16, 24, 32, 48, 64}
    for r in reqs:
        w = r.work
        assert w.n[0] == w.n[1] == w.n[2] and w.y_he == 0.0 and w.bins.n_bins == 1
        assert 1 <= len(w.src_ndot) <= 16 and w.steps == 5 and w.n_sub == 10
        assert w.packets % w.n_sub == 0 and w.packets // w.n_sub >= len(w.src_ndot)
        assert 0.9e4 <= w.packets <= 1.0e6
    uniform = sum(1 for r in reqs if np.all(r.work.n_h == r.work.n_h[0]))
    assert 200 < uniform < 312                              # uniform or lognormal, 50/50


def test_workspace_bytes_grow_with_the_grid():
    reqs = W.serving_stream(count=40, seed=5)
    by_side = {}
    for r in reqs:
        by_side.setdefault(r.work.n[0], []).append(serve.workspace_bytes(r.work, fp64=False))
    sides = sorted(by_side)
    means = [np.mean(by_side[s]) for s in sides]
    assert all(b > a for a, b in zip(means, means[1:]))
    r = reqs[0]
    assert serve.workspace_bytes(r.work, fp64=True) > serve.workspace_bytes(r.work, fp64=False)


class FakeExecutor:
    """Stands in for the GPU: a step 'costs' a fixed time on a fake clock."""

    def __init__(self, clock):
        self.clock = clock
        self.calls = []
        self.open_now = set()

    def open(self, work):
        h = object()
        self.open_now.add(h)
        return (h, work)

    def step(self, solves):
        self.calls.append([w.solve_id for _, w in solves])
        self.clock.t += 0.004
        return [dict(emitted=1.0, absorbed=0.5, escaped=0.5, truncated=0.0, crossings=10, packets=w.packets)
                for _, w in solves]

    def fetch(self, s):
        return None

    def close(self, s):
        self.open_now.remove(s[0])

    def release(self):
        pass


class FakeAsyncExecutor(FakeExecutor):
    """As FakeExecutor, with the call split into launch and wait (the server
    then opens the next requests while a call runs)."""

    def __init__(self, clock):
        super().__init__(clock)
        self.pending = None
        self.opened_during_call = 0

    def open(self, work):
        if self.pending is not None:
            self.opened_during_call += 1
        return super().open(work)

    def launch(self, solves):
        assert self.pending is None
        self.pending = solves

    def busy(self):
        return True

    def wait(self):
        solves, self.pending = self.pending, None
        return self.step(solves)


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-6
        return self.t


@pytest.mark.parametrize("overlap", [False, True], ids=["sync", "open-during-call"])
@pytest.mark.parametrize("slots,budget_solves", [(4, 100), (8, 3), (64, 1000)])
def test_continuous_batching_loop(slots, budget_solves, overlap, monkeypatch):
    reqs = W.serving_stream(count=30, seed=6, sides=(16, 24), log_packets=(4.0, 4.5), rate_per_s=500.0)
    need = {r.rid: serve.workspace_bytes(r.work, fp64=False) for r in reqs}
    budget = int(budget_solves * max(need.values()))
    clock = FakeClock()
    monkeypatch.setattr(serve.time, "sleep", lambda s: setattr(clock, "t", clock.t + s))
    ex = FakeAsyncExecutor(clock) if overlap else FakeExecutor(clock)
    srv = serve.Server(max_slots=slots, hbm_budget=budget, executor=ex, keep_fields=False)
    out = srv.run(reqs, clock=clock)
    if overlap and slots == 4:
        assert ex.opened_during_call > 0                    # requests in line went up during calls
    assert [o.rid for o in out] == [r.rid for r in reqs]
    assert not ex.open_now                                  # every solve closed
    steps = {}
    for call in ex.calls:
        assert len(call) <= slots and len(set(call)) == len(call)
        for sid in call:
            steps[sid] = steps.get(sid, 0) + 1
    assert all(steps[r.work.solve_id] == r.work.steps for r in reqs)
    assert srv.peak_bytes <= budget
    first_call = {}
    for k, call in enumerate(ex.calls):
        for sid in call:
            first_call.setdefault(sid, k)
    order = [first_call[r.work.solve_id] for r in reqs]
    assert order == sorted(order)                           # admitted in arrival order
    for o, r in zip(out, reqs):
        assert o.admit_s >= r.arrival_s - 1e-9 and o.done_s > o.admit_s and o.latency_s > 0
    if slots == 64 and budget_solves >= 30:
        # joins between calls: some call holds requests admitted at different calls
        assert any(len(c) > 1 for c in ex.calls)


def test_server_rejects_bad_limits():
    with pytest.raises(ValueError):
        serve.Server(max_slots=0, hbm_budget=1, executor=object())
    reqs = W.serving_stream(count=2, seed=7)
    srv = serve.Server(max_slots=2, hbm_budget=10, executor=FakeExecutor(FakeClock()))
    with pytest.raises(ValueError):
        srv.run(reqs)


def test_percentiles():
    v = list(range(1, 101))
    assert serve.percentile(v, 50) == pytest.approx(50.5, abs=0)
    assert serve.percentile(v, 99) == pytest.approx(99.01, abs=0)


def test_opened_ahead_requests_are_admitted_in_order(monkeypatch):
    """All present, two slots, room for every workspace: the requests opened
    during a call are the next ones in arrival order, and each is admitted
    (and closed) exactly once."""
    reqs = W.serving_stream(count=9, seed=8, sides=(16,), log_packets=(4.0, 4.2), rate_per_s=500.0)
    clock = FakeClock()
    monkeypatch.setattr(serve.time, "sleep", lambda s: setattr(clock, "t", clock.t + s))
    ex = FakeAsyncExecutor(clock)
    srv = serve.Server(max_slots=2, hbm_budget=1 << 40, executor=ex, keep_fields=False)
    out = srv.run(reqs, realtime=False, clock=clock)
    assert [o.rid for o in out] == [r.rid for r in reqs]
    assert not ex.open_now and ex.opened_during_call >= 2
    seen = []
    for call in ex.calls:
        for sid in call:
            if sid not in seen:
                seen.append(sid)
    assert seen == [r.work.solve_id for r in reqs]
    assert srv.peak_bytes <= 4 * max(serve.workspace_bytes(r.work, fp64=False) for r in reqs)


def test_a_failed_run_closes_its_solves(monkeypatch):
    """A request whose opening fails ends the run with its error, and every
    solve the run opened (admitted or opened ahead) is closed again."""
    reqs = W.serving_stream(count=6, seed=9, sides=(16,), log_packets=(4.0, 4.2), rate_per_s=500.0)
    clock = FakeClock()
    monkeypatch.setattr(serve.time, "sleep", lambda s: setattr(clock, "t", clock.t + s))

    class Failing(FakeAsyncExecutor):
        def open(self, work):
            if work.solve_id == reqs[3].work.solve_id:
                raise RuntimeError("no memory")
            return super().open(work)

    ex = Failing(clock)
    srv = serve.Server(max_slots=2, hbm_budget=1 << 40, executor=ex, keep_fields=False)
    with pytest.raises(RuntimeError):
        srv.run(reqs, realtime=False, clock=clock)
    assert not ex.open_now


def test_backlog_is_opened_while_calls_run(monkeypatch):
    """All present, a backlog longer than sync_open: only sync_open requests
    are opened before the first call; once the batch is half full every later
    one goes up while a call runs, and all are served in arrival order."""
    reqs = W.serving_stream(count=40, seed=10, sides=(16,), log_packets=(4.0, 4.2), rate_per_s=500.0)
    clock = FakeClock()
    monkeypatch.setattr(serve.time, "sleep", lambda s: setattr(clock, "t", clock.t + s))

    class Counting(FakeAsyncExecutor):
        opened_between_calls = 0

        def open(self, work):
            if self.pending is None:
                self.opened_between_calls += 1
            return super().open(work)

    ex = Counting(clock)
    srv = serve.Server(max_slots=16, hbm_budget=1 << 40, executor=ex, keep_fields=False, sync_open=4)
    out = srv.run(reqs, realtime=False, clock=clock)
    assert [o.rid for o in out] == [r.rid for r in reqs]
    assert not ex.open_now
    assert len(ex.calls[0]) == 4
    assert ex.opened_between_calls <= 8 and ex.opened_during_call >= len(reqs) - 8
    assert max(len(c) for c in ex.calls) == 16


def test_server_rejects_a_zero_sync_open():
    with pytest.raises(ValueError):
        serve.Server(max_slots=4, hbm_budget=1 << 30, executor=FakeExecutor(FakeClock()), sync_open=0)
