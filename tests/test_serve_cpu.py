"""The serving scheduler on a CPU fake executor: admission by HBM budget, continuous batching,
retirement, failure isolation and the sequential baseline (no GPU)."""

import pytest

from paper_2502_10872_amd import serve as V


def reqs(sizes, steps=3, gap=0.0):
    return [V.Request(rid=k, t_arrival=k * gap, spec=dict(n=n, model="SS", radius=1.0, seed=k), steps=steps)
            for k, n in enumerate(sizes)]


def test_all_requests_complete_in_batches():
    cfg = V.ServeConfig(hbm_budget=1 << 40, builders=2)
    ex = V.FakeExecutor(cfg, sleep=False)
    rs = reqs([40, 60, 80, 100, 120], steps=4)
    out = V.Server(ex, cfg).run(rs, realtime=False)
    assert out["completed"] == 5 and out["rejected"] == 0 and out["failed"] == 0
    assert all(r.steps_done == 4 for r in rs)
    assert max(len(b) for b in ex.batches) >= 2  # requests shared ticks
    assert all(r.t_done >= r.t_ready >= r.t_admit >= r.t_arrival for r in rs)


def test_hbm_budget_bounds_resident_footprint():
    cfg = V.ServeConfig(hbm_budget=int(1100 * 3 * 100 ** 2), builders=3)
    ex = V.FakeExecutor(cfg, sleep=False)
    rs = reqs([100] * 10, steps=2)
    server = V.Server(ex, cfg)
    out = server.run(rs, realtime=False)
    assert out["completed"] == 10
    assert server.max_in_use <= cfg.hbm_budget
    assert max(len(b) for b in ex.batches) <= 3


def test_oversized_and_overflow_requests_are_rejected():
    cfg = V.ServeConfig(hbm_budget=int(1100 * 50 ** 2), max_queue=2, builders=1)
    ex = V.FakeExecutor(cfg, sleep=False)
    rs = reqs([60, 10, 10, 10, 10, 10], steps=1)  # the first can never fit; the queue holds two
    out = V.Server(ex, cfg).run(rs, realtime=False)
    assert rs[0].status == "rejected"
    assert out["rejected"] >= 1 and out["completed"] + out["rejected"] == 6


def test_failed_build_retires_alone():
    cfg = V.ServeConfig(hbm_budget=1 << 40, builders=2)
    ex = V.FakeExecutor(cfg, sleep=False, fail=lambda r: r.rid == 2)
    rs = reqs([30, 30, 30, 30], steps=2)
    out = V.Server(ex, cfg).run(rs, realtime=False)
    assert rs[2].status == "failed" and out["failed"] == 1 and out["completed"] == 3


def test_nonfinite_mesh_retires_alone():
    """A mesh whose state goes non-finite (reported in its own step stats) retires as failed after that
    step, in the continuous server and one at a time; the other requests complete."""
    cfg = V.ServeConfig(hbm_budget=1 << 40, builders=2)
    rs = reqs([30, 30, 30, 30], steps=3)
    out = V.Server(V.FakeExecutor(cfg, sleep=False, diverge=lambda r: r.rid == 1), cfg).run(rs, realtime=False)
    assert rs[1].status == "failed" and rs[1].steps_done == 2 and rs[1].error == "non-finite state"
    assert out["failed"] == 1 and out["completed"] == 3
    rs2 = reqs([30, 30, 30, 30], steps=3)
    seq = V.run_sequential(V.FakeExecutor(cfg, sleep=False, diverge=lambda r: r.rid == 1), cfg, rs2, realtime=False)
    assert rs2[1].status == "failed" and rs2[1].steps_done == 2
    assert seq["failed"] == 1 and seq["completed"] == 3


def test_realtime_latency_accounting_and_sequential_baseline():
    cfg = V.ServeConfig(hbm_budget=1 << 40, builders=2)
    # steps (20 ms per mesh) outlast the arrival gap (5 ms), so later arrivals join running batches
    rs = reqs([100, 100, 100, 100], steps=3, gap=0.005)
    out = V.Server(V.FakeExecutor(cfg, step_s_per_vertex=2e-6), cfg).run(rs)
    assert out["completed"] == 4 and out["p99_s"] >= out["p50_s"] > 0
    rs2 = reqs([100, 100, 100, 100], steps=3, gap=0.005)
    seq = V.run_sequential(V.FakeExecutor(cfg, step_s_per_vertex=2e-6), cfg, rs2)
    assert seq["completed"] == 4
    # batching amortises the per-step overhead: fewer ticks than the sequential path's steps
    assert out["ticks"] < 12


def test_requests_past_the_wait_deadline_are_shed():
    # one slot, 30 ms per step, 4 steps per request: the queue outgrows a 50 ms wait deadline
    cfg = V.ServeConfig(hbm_budget=1 << 40, builders=1, max_active=1, max_wait_s=0.05)
    rs = reqs([100] * 6, steps=4, gap=0.002)
    out = V.Server(V.FakeExecutor(cfg, step_s_per_vertex=3e-6), cfg).run(rs)
    assert out["shed"] >= 1 and out["completed"] >= 1
    assert out["completed"] + out["shed"] == 6 and out["rejected"] == 0
    assert all(r.steps_done == 0 for r in rs if r.status == "shed")
    # the one-at-a-time path sheds by the same deadline
    rs2 = reqs([100] * 6, steps=4, gap=0.002)
    seq = V.run_sequential(V.FakeExecutor(cfg, step_s_per_vertex=3e-6), cfg, rs2)
    assert seq["shed"] >= 1 and seq["completed"] + seq["shed"] == 6
