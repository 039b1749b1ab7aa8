"""Admission logic of the serving loop, with a host-only runner."""
import threading
import time

import numpy as np

from paper_1705_05784_amd.serving import Server, summarize


class _Req:
    def __init__(self, rid, arrival, cost, mem):
        self.rid, self.arrival, self.cost, self.mem = rid, arrival, cost, mem


class _Runner:
    def __init__(self):
        self.lock = threading.Lock()
        self.inflight = 0
        self.mem = 0
        self.peak = 0
        self.peak_mem = 0
        self.order = []

    def __call__(self, req, res):
        with self.lock:
            self.inflight += 1
            self.mem += req.mem
            self.peak = max(self.peak, self.inflight)
            self.peak_mem = max(self.peak_mem, self.mem)
            self.order.append(req.rid)
        time.sleep(req.cost)
        res.iterations.append(3)
        with self.lock:
            self.inflight -= 1
            self.mem -= req.mem


def test_slots_and_budget_respected():
    rng = np.random.default_rng(0)
    reqs = [_Req(i, 0.0, float(rng.uniform(0.005, 0.02)), int(rng.integers(1, 5))) for i in range(24)]
    run = _Runner()
    srv = Server(run, slots=4, hbm_budget=8, footprint=lambda r: r.mem)
    res = srv.run(reqs, realtime=False)
    assert all(r.status == 0 for r in res)
    assert run.peak <= 4 and srv.peak_inflight <= 4
    assert run.peak_mem <= 8 and srv.peak_reserved <= 8
    assert run.peak >= 2                      # requests overlapped
    assert run.order == sorted(run.order)     # first come, first served
    s = summarize(res)
    assert s["solves"] == 24 and s["p99_s"] >= s["p50_s"] > 0


def test_oversized_request_rejected_others_served():
    reqs = [_Req(0, 0.0, 0.001, 2), _Req(1, 0.0, 0.001, 100), _Req(2, 0.0, 0.001, 2)]
    srv = Server(_Runner(), slots=2, hbm_budget=10, footprint=lambda r: r.mem)
    res = srv.run(reqs, realtime=False)
    assert [r.status for r in res] == [0, -6, 0]
    assert "exceeds budget" in res[1].error


def test_arrivals_are_honoured():
    reqs = [_Req(i, 0.02 * i, 0.001, 1) for i in range(5)]
    srv = Server(_Runner(), slots=2, hbm_budget=10, footprint=lambda r: r.mem)
    res = srv.run(reqs, realtime=True)
    for r in res:
        assert r.t_admit >= r.t_arrival - 1e-6
        assert r.t_done >= r.t_admit
        assert r.latency < 0.5


def test_runner_failure_is_reported():
    def bad(req, res):
        raise RuntimeError("boom")
    srv = Server(bad, slots=2, hbm_budget=10, footprint=lambda r: 1)
    res = srv.run([_Req(0, 0.0, 0.0, 1)], realtime=False)
    assert res[0].status == -1 and "boom" in res[0].error


def test_in_process_runner_is_single_slot():
    import pytest

    from paper_1705_05784_amd.serving import GpuRunner
    srv = Server(GpuRunner(0), slots=2, hbm_budget=10, footprint=lambda r: 1)
    with pytest.raises(ValueError):
        srv.run([_Req(0, 0.0, 0.0, 1)], realtime=False)
