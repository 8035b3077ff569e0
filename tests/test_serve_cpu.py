"""The serving scheduler on a fake executor and a fake clock (no GPU): FIFO
admission by footprint and slots, continuous batching, eviction on steady /
non-finite / step cap, refusal of requests larger than the budget, and the
latency statistics."""
import pytest

from paper_2312_00369_amd.serve import Executor, Server, percentile


class FakeExecutor(Executor):
    """Case k becomes steady after steps_to_steady[k] steps; a step of the whole
    batch costs `step_cost` seconds of fake time per chunk regardless of size
    (batching), and every admitted case advances together."""

    def __init__(self, step_cost=1.0, nonfinite=()):
        self.t = 0.0
        self.step_cost = step_cost
        self.live = {}
        self.nonfinite = set(nonfinite)
        self.log = []
        self._next = 0

    def now(self):
        return self.t

    def wait_until(self, t):
        self.t = max(self.t, t)

    def footprint(self, req):
        return req["fp"]

    def admit(self, req):
        k = self._next
        self._next += 1
        self.live[k] = dict(req=req, steps=0)
        self.log.append(("admit", req["id"], self.t))
        return k

    def step(self, n):
        for v in self.live.values():
            v["steps"] += n
        self.t += self.step_cost
        self.log.append(("step", len(self.live), self.t))

    def poll(self):
        out = {}
        for k, v in self.live.items():
            r = v["req"]
            out[k] = dict(steady=v["steps"] >= r["to_steady"],
                          nonfinite=r["id"] in self.nonfinite and v["steps"] >= 1000,
                          steps=v["steps"], theta_deg=90.0, mass=1.0)
        return out

    def release(self, k):
        v = self.live.pop(k)
        self.log.append(("release", v["req"]["id"], self.t))
        return dict(steps=v["steps"])


def _req(i, arrival, fp, to_steady):
    return dict(id=i, arrival_s=arrival, fp=fp, to_steady=to_steady, shape=(10, 10))


def test_continuous_batching_and_latency():
    reqs = [_req(0, 0.0, 4, 3000), _req(1, 0.5, 4, 1000), _req(2, 0.6, 4, 2000),
            _req(3, 5.0, 4, 1000)]
    ex = FakeExecutor()
    rec, summ = Server(ex, budget_bytes=8, max_slots=8, chunk_steps=1000).run(reqs)
    # request 1 arrives while 0 runs and is admitted at the next boundary (t = 1)
    admits = {e[1]: e[2] for e in ex.log if e[0] == "admit"}
    assert admits[0] == 0.0 and admits[1] == 1.0
    # request 2 waits for memory: budget 8 holds two cases; 1 leaves at t = 2
    assert admits[2] == 2.0
    assert all(r["steady"] for r in rec)
    assert rec[1]["time_to_steady_s"] == pytest.approx(2.0 - 0.5)
    assert rec[3]["admit_s"] == 5.0
    assert summ["served"] == 4 and summ["steady"] == 4
    assert summ["p50_time_to_steady_s"] == pytest.approx(
        percentile([r["time_to_steady_s"] for r in rec], 50))
    # batching: while two cases are resident they advance in the same step
    assert any(e[0] == "step" and e[1] == 2 for e in ex.log)


def test_slots_limit_and_fifo():
    reqs = [_req(i, 0.0, 1, 1000 * (i + 1)) for i in range(5)]
    ex = FakeExecutor()
    rec, _ = Server(ex, budget_bytes=100, max_slots=2, chunk_steps=1000).run(reqs)
    order = [e[1] for e in ex.log if e[0] == "admit"]
    assert order == [0, 1, 2, 3, 4]
    assert max(e[1] for e in ex.log if e[0] == "step") <= 2


def test_refusal_nonfinite_and_step_cap():
    reqs = [_req(0, 0.0, 50, 1000), _req(1, 0.0, 2, 10 ** 9), _req(2, 0.0, 2, 10 ** 9)]
    ex = FakeExecutor(nonfinite={2})
    rec, summ = Server(ex, budget_bytes=10, max_slots=4, chunk_steps=1000,
                       max_steps=5000).run(reqs)
    assert "refused" in rec[0]
    assert rec[1]["status"] == "step cap" and rec[1]["steps"] == 5000
    assert rec[2]["status"] == "nonfinite"
    assert summ["refused"] == 1 and summ["steady"] == 0


def test_percentile():
    assert percentile([1, 2, 3, 4], 50) == 2.5
    assert percentile([5], 99) == 5
    assert percentile([], 50) is None


def test_per_request_cap_and_time_to_result():
    """A request's own max_steps overrides the server cap; time-to-result covers
    every case that left, time-to-steady only the steady ones; per-lattice
    counts split steady from capped."""
    reqs = [_req(0, 0.0, 1, 10 ** 9), _req(1, 0.0, 1, 2000), _req(2, 0.0, 1, 10 ** 9)]
    reqs[0]["max_steps"] = 3000
    reqs[2]["lattice"] = "D3Q19"
    ex = FakeExecutor()
    rec, summ = Server(ex, budget_bytes=10, max_slots=4, chunk_steps=1000,
                       max_steps=6000).run(reqs)
    assert rec[0]["status"] == "step cap" and rec[0]["steps"] == 3000
    assert rec[1]["status"] == "steady" and rec[1]["steps"] == 2000
    assert rec[2]["status"] == "step cap" and rec[2]["steps"] == 6000
    assert rec[0]["time_to_result_s"] == pytest.approx(3.0)
    assert rec[1]["time_to_result_s"] == pytest.approx(rec[1]["time_to_steady_s"])
    assert "time_to_steady_s" not in rec[0]
    assert summ["p99_time_to_result_s"] == pytest.approx(percentile([3.0, 2.0, 6.0], 99))
    assert summ["by_lattice"]["D2Q9"] == dict(requests=2, steady=1, capped=1, nonfinite=0)
    assert summ["by_lattice"]["D3Q19"] == dict(requests=1, steady=0, capped=1, nonfinite=0)
    assert summ["utilisation"] == pytest.approx(1.0)


def test_chunks_never_pass_a_step_cap():
    """A cap that is not a multiple of the chunk: the last chunk is shortened,
    so the capped case stops exactly at its cap (the others advance with it)."""
    reqs = [_req(0, 0.0, 1, 10 ** 9), _req(1, 0.0, 1, 10 ** 9)]
    reqs[0]["max_steps"] = 2500
    ex = FakeExecutor()
    rec, _ = Server(ex, budget_bytes=10, max_slots=4, chunk_steps=1000,
                    max_steps=4000).run(reqs)
    assert rec[0]["status"] == "step cap" and rec[0]["steps"] == 2500
    assert rec[1]["status"] == "step cap" and rec[1]["steps"] == 4000
