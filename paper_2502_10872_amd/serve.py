"""Continuous-batching server for implicit-step requests on one GPU.

A request brings a mesh (size, model, rest curvature) and asks for a number of implicit steps.  The
server keeps every admitted request's stencils, constant Hessian and state resident in HBM and advances
all of them together: each tick is one batched implicit step (one launch per phase over every active
mesh, per-mesh Newton and PCG control), and requests join and leave between ticks:

* arrival      -> FIFO queue (bounded; a request whose estimated footprint can never fit is rejected)
* shedding     -> a request still queued max_wait_s after its arrival is dropped (status "shed")
* admission    -> while the HBM budget and the slot limit allow, the queue head is handed to a builder
                  thread (topology, rest precompute and Hessian assembly on the builder's own stream)
* ready        -> joins the active batch at the next tick
* done         -> after its last step the request retires and its memory is released

Latency is arrival -> completion.  `run_sequential` serves the same trace one mesh at a time, for
comparison.  Executors: `GpuExecutor` (the HIP library) and `FakeExecutor` (a CPU model of costs, for
testing the scheduler without a GPU).
"""

from __future__ import annotations

import argparse
import collections
import concurrent.futures as cf
import json
import math
import sys
import threading
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    t_arrival: float
    spec: dict
    steps: int = 10
    nv: int = 0
    est_bytes: int = 0
    bytes: int = 0
    t_admit: float = math.nan
    t_ready: float = math.nan
    t_done: float = math.nan
    steps_done: int = 0
    newton: int = 0
    pcg: int = 0
    status: str = "queued"
    handle: object = None
    error: str = ""
    result: object = None


@dataclass
class ServeConfig:
    hbm_budget: int = 16 << 30
    max_active: int = 256
    max_queue: int = 100000
    max_wait_s: float = math.inf  # queue-wait deadline: longer-waiting requests are shed
    builders: int = 4
    dt: float = 1.0 / 60.0
    max_newton: int = 4
    pcg_rtol: float = 1e-2
    max_pcg: int = 100000
    precision: int = 1  # mixed
    bytes_per_vertex: float = 1500.0  # a-priori footprint per vertex; raised to the largest measured ratio
    keep_state: bool = False  # keep each request's final positions (for tests)


class GpuExecutor:
    """Builds requests with the HIP library and steps the active set as one batch."""

    def __init__(self, cfg: ServeConfig, device: int = 0):
        import torch

        from . import inputs as I
        from . import shell as S

        self.S, self.I, self.torch = S, I, torch
        self.cfg = cfg
        torch.cuda.set_device(device)
        self.stream = torch.cuda.Stream()
        self.batch = None
        self._local = threading.local()
        self.params, self._keep = S.step_params(cfg.dt, gravity=I.GRAVITY, max_newton=cfg.max_newton,
                                                max_pcg=cfg.max_pcg, pcg_rtol=cfg.pcg_rtol)

    def mesh(self, spec):
        return self.I.mesh_from_spec(spec, spacing=0.01)

    def build(self, req: Request):
        torch = self.torch
        if not hasattr(self._local, "stream"):
            self._local.stream = torch.cuda.Stream()
        mesh = self.mesh(req.spec)
        S = self.S
        st = S.shell_build_stencils(mesh.X, mesh.tris, mesh.model, self.I.MATERIAL, self.cfg.precision,
                                    stream=self._local.stream)
        h = S.shell_assemble_constant_hessian(st, stream=self._local.stream)
        sim = S.shell_sim_create(st, h, mesh.X, None, mesh.pinned)
        req.bytes = S.shell_sim_device_bytes(sim)
        return (st, h, sim, mesh)

    def step(self, reqs):
        S = self.S
        sims = [r.handle[2] for r in reqs]
        if self.batch is None:
            self.batch = S.shell_batch_create(sims)
        else:
            S.shell_batch_reset(self.batch, sims)
        # a mesh whose state went non-finite is reported in its own stats; the others stepped normally
        rc, stats = S.shell_batch_step(self.batch, self.params, len(sims), stream=self.stream, allow_nonfinite=True)
        return stats

    def state(self, req):
        st, h, sim, mesh = req.handle
        return self.S.shell_sim_get_state(sim, mesh.nv)

    def release(self, req):
        st, h, sim, mesh = req.handle
        if self.cfg.keep_state:
            req.result = self.S.shell_sim_get_state(sim, mesh.nv)[0]
        self.S.shell_destroy_sim(sim)
        self.S.shell_destroy_hessian(h)
        self.S.shell_destroy_stencils(st)
        req.handle = None

    def close(self):
        if self.batch is not None:
            self.S.shell_destroy_batch(self.batch)
            self.batch = None


class FakeExecutor:
    """CPU stand-in with a cost model: build time and per-step time linear in the vertex count, a
    batch step costing a launch overhead plus the sum of the members' work.  Tests the scheduler."""

    def __init__(self, cfg: ServeConfig, build_s_per_vertex=2e-8, step_s_per_vertex=5e-9, step_overhead=1e-4,
                 sleep=True, fail=None, diverge=None):
        self.cfg = cfg
        self.bspv, self.sspv, self.ovh, self.sleep = build_s_per_vertex, step_s_per_vertex, step_overhead, sleep
        self.fail = fail or (lambda req: False)
        self.diverge = diverge or (lambda req: False)  # requests whose state goes non-finite at their 2nd step
        self.batches = []

    def build(self, req):
        if self.fail(req):
            raise RuntimeError("injected build failure")
        if self.sleep:
            time.sleep(self.bspv * req.nv)
        req.bytes = int(self.cfg.bytes_per_vertex * 0.9 * req.nv)
        return ("fake", req.nv)

    def step(self, reqs):
        self.batches.append([r.rid for r in reqs])
        if self.sleep:
            time.sleep(self.ovh + self.sspv * sum(r.nv for r in reqs))
        return [dict(newton_iters=2, pcg_total=60, status=5 if self.diverge(r) and r.steps_done == 1 else 0)
                for r in reqs]

    def release(self, req):
        req.handle = None

    def close(self):
        pass


def nv_of(spec) -> int:
    return int(spec["n"]) ** 2


def percentile(values, q):
    return float(np.percentile(np.asarray(values), q)) if len(values) else math.nan


class Server:
    def __init__(self, executor, cfg: ServeConfig):
        self.ex = executor
        self.cfg = cfg
        self.in_use = 0
        self.max_in_use = 0
        self.bpv = cfg.bytes_per_vertex
        self.ticks = 0
        self.batch_sizes = []

    def _estimate(self, req):
        req.nv = nv_of(req.spec)
        req.est_bytes = int(self.bpv * req.nv)

    def run(self, requests, realtime=True):
        """Serve `requests` (sorted by arrival).  realtime: arrivals follow the wall clock from the start;
        otherwise all requests are present at time 0."""
        cfg = self.cfg
        for r in requests:
            self._estimate(r)
        queue = collections.deque()
        building = {}
        active = []
        done = []
        nxt = 0
        pool = cf.ThreadPoolExecutor(max_workers=cfg.builders)
        t0 = time.perf_counter()
        clock = (lambda: time.perf_counter() - t0)
        try:
            while len(done) < len(requests):
                now = clock()
                while nxt < len(requests) and (not realtime or requests[nxt].t_arrival <= now):
                    r = requests[nxt]
                    nxt += 1
                    if not realtime:
                        r.t_arrival = 0.0
                    if r.est_bytes > cfg.hbm_budget or len(queue) >= cfg.max_queue:
                        r.status = "rejected"
                        r.t_done = now
                        done.append(r)
                    else:
                        queue.append(r)
                # shedding: requests that waited past the deadline leave the queue unserved
                if queue and now - queue[0].t_arrival > cfg.max_wait_s:
                    kept = collections.deque()
                    for r in queue:
                        if now - r.t_arrival > cfg.max_wait_s:
                            r.status = "shed"
                            r.t_done = now
                            done.append(r)
                        else:
                            kept.append(r)
                    queue = kept
                # admission: FIFO under the HBM budget and the slot limit
                while queue and len(building) + len(active) < cfg.max_active and \
                        self.in_use + int(self.bpv * queue[0].nv) <= cfg.hbm_budget:
                    r = queue.popleft()
                    r.est_bytes = int(self.bpv * r.nv)
                    r.t_admit = clock()
                    r.status = "building"
                    self.in_use += r.est_bytes
                    self.max_in_use = max(self.max_in_use, self.in_use)
                    building[pool.submit(self.ex.build, r)] = r
                # finished builds join the batch
                for fut in [f for f in building if f.done()]:
                    r = building.pop(fut)
                    try:
                        r.handle = fut.result()
                    except Exception as e:  # a failed build retires alone; the others continue
                        r.status = "failed"
                        r.error = str(e)
                        r.t_done = clock()
                        self.in_use -= r.est_bytes
                        done.append(r)
                        continue
                    self.in_use += r.bytes - r.est_bytes
                    self.max_in_use = max(self.max_in_use, self.in_use)
                    # admission estimates follow the largest footprint per vertex seen so far
                    self.bpv = max(self.bpv, r.bytes / max(r.nv, 1))
                    r.t_ready = clock()
                    r.status = "active"
                    active.append(r)
                if active:
                    stats = self.ex.step(active)
                    self.ticks += 1
                    self.batch_sizes.append(len(active))
                    t = clock()
                    keep = []
                    for r, s in zip(active, stats):
                        r.steps_done += 1
                        r.newton += int(s["newton_iters"])
                        r.pcg += int(s["pcg_total"])
                        if s.get("status", 0) == 5:
                            r.status = "failed"
                            r.error = "non-finite state"
                        if r.steps_done >= r.steps or r.status == "failed":
                            if r.status != "failed":
                                r.status = "done"
                            r.t_done = t
                            self.ex.release(r)
                            self.in_use -= r.bytes
                            done.append(r)
                        else:
                            keep.append(r)
                    active = keep
                elif building:
                    cf.wait(list(building), timeout=0.05, return_when=cf.FIRST_COMPLETED)
                elif nxt < len(requests):
                    time.sleep(max(0.0, min(0.05, requests[nxt].t_arrival - clock())))
        finally:
            pool.shutdown(wait=True)
            self.ex.close()
        return summarize(requests, clock(), self)


def run_sequential(executor, cfg: ServeConfig, requests, realtime=True):
    """The same trace served one mesh at a time: build, then all its steps alone, FIFO."""
    for r in requests:
        r.nv = nv_of(r.spec)
    t0 = time.perf_counter()
    clock = (lambda: time.perf_counter() - t0)
    try:
        for r in requests:
            if realtime:
                wait = r.t_arrival - clock()
                if wait > 0:
                    time.sleep(wait)
            else:
                r.t_arrival = 0.0
            if clock() - r.t_arrival > cfg.max_wait_s:
                r.status, r.t_done = "shed", clock()
                continue
            r.t_admit = clock()
            try:
                r.handle = executor.build(r)
            except Exception as e:
                r.status, r.error, r.t_done = "failed", str(e), clock()
                continue
            r.t_ready = clock()
            r.status = "done"
            for _ in range(r.steps):
                s = executor.step([r])[0]
                r.steps_done += 1
                r.newton += int(s["newton_iters"])
                r.pcg += int(s["pcg_total"])
                if s.get("status", 0) == 5:
                    r.status, r.error = "failed", "non-finite state"
                    break
            r.t_done = clock()
            executor.release(r)
    finally:
        executor.close()
    return summarize(requests, clock(), None)


def summarize(requests, wall, server):
    ok = [r for r in requests if r.status == "done"]
    lat = [r.t_done - r.t_arrival for r in ok]
    qd = [r.t_admit - r.t_arrival for r in ok]
    steps = sum(r.steps_done for r in ok)
    out = dict(requests=len(requests), completed=len(ok),
               rejected=sum(r.status == "rejected" for r in requests),
               shed=sum(r.status == "shed" for r in requests),
               failed=sum(r.status == "failed" for r in requests),
               wall_s=wall, req_per_s=len(ok) / wall if wall > 0 else math.nan,
               steps_per_s=steps / wall if wall > 0 else math.nan,
               p50_s=percentile(lat, 50), p99_s=percentile(lat, 99),
               queue_p50_s=percentile(qd, 50), queue_p99_s=percentile(qd, 99),
               mean_nv=float(np.mean([r.nv for r in ok])) if ok else math.nan)
    if server is not None:
        out.update(ticks=server.ticks, mean_batch=float(np.mean(server.batch_sizes)) if server.batch_sizes else 0.0,
                   max_batch=int(max(server.batch_sizes)) if server.batch_sizes else 0, max_hbm_bytes=server.max_in_use)
    return out


def make_requests(rate, duration, seed=2502108725, steps=10, nv_max=1e6):
    from . import inputs as I

    trace = I.serving_trace(rate=rate, duration=duration, seed=seed, nv_max=nv_max)
    return [Request(rid=k, t_arrival=t["t"], spec=dict(n=t["n"], model=t["model"], radius=t["radius"],
                                                      seed=t["seed"]), steps=steps) for k, t in enumerate(trace)]


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--rates", default="5,20,50,100,200")
    ap.add_argument("--duration", type=float, default=4.0, help="seconds of arrivals per rate")
    ap.add_argument("--budget-gb", type=float, default=16.0)
    ap.add_argument("--builders", type=int, default=4)
    ap.add_argument("--nv-max", type=float, default=1e6)
    ap.add_argument("--sequential", action="store_true", help="also serve each trace one mesh at a time")
    ap.add_argument("--max-wait", type=float, default=math.inf, help="queue-wait deadline past which a request is shed")
    args = ap.parse_args(argv)
    cfg = ServeConfig(hbm_budget=int(args.budget_gb * (1 << 30)), builders=args.builders, max_wait_s=args.max_wait)
    results = []
    for rate in [float(r) for r in args.rates.split(",")]:
        reqs = make_requests(rate, args.duration, nv_max=args.nv_max)
        res = Server(GpuExecutor(cfg), cfg).run(reqs)
        res.update(mode="continuous", rate=rate)
        print(json.dumps(res), flush=True)
        results.append(res)
        if args.sequential:
            reqs = make_requests(rate, args.duration, nv_max=args.nv_max)
            res = run_sequential(GpuExecutor(cfg), cfg, reqs)
            res.update(mode="sequential", rate=rate)
            print(json.dumps(res), flush=True)
            results.append(res)
    return results


if __name__ == "__main__":
    main(sys.argv[1:])
