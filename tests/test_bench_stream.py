"""Host-side logic of the served-stream harness (bench.py's _StreamRun) on a fake
context: jobs are submitted in index order, every job is collected once, and the
host-byte window never deadlocks when a large job follows small ones under open-loop
arrivals (later jobs must not take the room an earlier job waits for)."""
import collections
import threading
import types

import pytest

import bench
from paper_1609_04567_amd import inputs as I


class _FakeCtx:
    """Completes every job at once, in submission order."""

    def __init__(self):
        self.cv = threading.Condition()
        self.done = collections.deque()
        self.order = []
        self.next_id = 1

    def submit_host(self, grid, stencil_id, reduce_op, cond, max_iter, bc, env0=None, param=()):
        with self.cv:
            jid = self.next_id
            self.next_id += 1
            self.order.append(grid)
            self.done.append(jid)
            self.cv.notify_all()
            return jid

    def wait_any(self, wait):
        with self.cv:
            self.cv.wait_for(lambda: self.done, timeout=30)
            return self.done.popleft()

    def result(self, jid):
        return types.SimpleNamespace(status=0)

    def stats(self):
        return {}


def _specs(sides):
    return [I.JobSpec(index=k, kind=I.KIND_LIFE, side=s, seed=k, arrival_u=0.5)
            for k, s in enumerate(sides)]


@pytest.mark.timeout(60)
@pytest.mark.parametrize("open_loop", [False, True])
def test_stream_keeps_order_and_window_without_deadlock(monkeypatch, open_loop):
    # byte window of 3 jobs of side 10; every fourth job fills the window alone
    sides = [10, 10, 10, 17] * 12
    specs = _specs(sides)
    kw = dict(stencil_id=0, reduce_op=0, cond=None, max_iter=1, bc=0)
    monkeypatch.setattr(bench, "_make_host_job", lambda L, I_, torch, spec, f32: (spec.index, None, kw))
    peak = [0]
    checked = []

    def check(k, v, job, r):
        checked.append(k)

    ctx = _FakeCtx()
    arrivals = [0.002 * k for k in range(len(specs))] if open_loop else None
    run = bench._StreamRun(None, I, None, ctx, specs, True, 300, arrivals=arrivals, check=check)
    orig = run._finish

    def finish(*a):
        with run.cv:
            peak[0] = max(peak[0], run.out_bytes)
        orig(*a)

    run._finish = finish
    run.run()
    assert ctx.order == list(range(len(specs)))
    assert sorted(checked) == list(range(len(specs)))
    assert run.out_bytes == 0
    assert peak[0] <= 300
