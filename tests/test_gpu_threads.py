"""Distinct handles driven from distinct host threads.

The library holds no state shared between handles: a simulation, a batch and their graphs belong to the
thread that drives them.  Two threads, each stepping its own batch on its own stream (resetting its member
list before every step, as a serving loop does, so that graphs are captured and released concurrently),
must reach bit for bit the states that the same sequences reach one after the other."""

import threading

import numpy as np
import pytest

from paper_2502_10872_amd import inputs as I
from paper_2502_10872_amd import shell as S

pytestmark = pytest.mark.gpu


def _meshes(lane):
    if lane == 0:
        return [I.plate_mesh(48, model="EP"), I.cylinder_mesh(40, model="FS"), I.plate_mesh(33, model="SP"),
                I.cylinder_mesh(64, model="SS")]
    return [I.sphere_cap_mesh(96, 1.5, model="SS"), I.cylinder_mesh(72, model="ES"), I.plate_mesh(57, model="FP")]


def _schedule(n, steps):
    """The members of each step: every mesh in the first, then subsets that change from step to step."""
    out = [list(range(n))]
    for k in range(1, steps):
        out.append([m for m in range(n) if (m + k) % 3 != 0] or [0])
    return out


def _run_lane(lane, torch, steps, out, errors):
    try:
        probs = [S.Problem(m, I.MATERIAL) for m in _meshes(lane)]
        stream = torch.cuda.Stream()
        params, _keep = S.step_params(1 / 60, max_newton=2, pcg_rtol=1e-6)
        batch = None
        try:
            for members in _schedule(len(probs), steps):
                sims = [probs[m].sim for m in members]
                if batch is None:
                    batch = S.shell_batch_create(sims)
                else:
                    S.shell_batch_reset(batch, sims)
                S.shell_batch_step(batch, params, len(sims), stream=stream)
            out[lane] = [S.shell_sim_get_state(pb.sim, pb.nv)[:2] for pb in probs]
        finally:
            if batch is not None:
                S.shell_destroy_batch(batch)
            for pb in probs:
                pb.close()
    except BaseException as e:  # reported by the main thread
        errors.append((lane, e))


def test_two_threads_stepping_their_own_batches_match_one_thread():
    import torch

    steps = 6
    seq = [None, None]
    errors = []
    for lane in (0, 1):
        _run_lane(lane, torch, steps, seq, errors)
    assert not errors, errors
    par = [None, None]
    threads = [threading.Thread(target=_run_lane, args=(lane, torch, steps, par, errors)) for lane in (0, 1)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=240)
    assert not any(t.is_alive() for t in threads)
    assert not errors, errors
    for lane in (0, 1):
        for (xs, vs), (xp, vp) in zip(seq[lane], par[lane]):
            assert np.isfinite(xp).all()
            assert np.array_equal(xs, xp) and np.array_equal(vs, vp)


def _reader(torch, done, counts, errors):
    """Builds, exports, reads and frees small problems (allocations, releases, host copies) until the
    stepping thread is done."""
    try:
        k = 0
        while not done.is_set() and k < 400:
            with S.Problem(I.plate_mesh(12 + k % 5, model="SS" if k % 2 else "EP"), I.MATERIAL) as pb:
                S.shell_stencils_export(pb.st)
                S.shell_hessian_export_csr(pb.h, pb.nv)
                x, v = S.shell_sim_get_state(pb.sim, pb.nv)[:2]
                S.shell_sim_set_state(pb.sim, x, v, 0)
                S.shell_sim_set_held(pb.sim, np.asarray(pb.mesh.pinned, dtype=np.uint8) * 7)
            k += 1
        counts.append(k)
    except BaseException as e:
        errors.append(("reader", e))


def test_host_calls_of_one_thread_leave_another_threads_graph_captures_intact():
    """One thread steps a batch whose member list changes every step (a graph is captured at each step)
    while another creates, exports, reads, writes and frees problems of its own: neither call fails, and
    the stepping thread reaches bit for bit the states it reaches alone."""
    import torch

    steps = 6
    alone = [None, None]
    errors = []
    _run_lane(1, torch, steps, alone, errors)
    assert not errors, errors
    together = [None, None]
    done = threading.Event()
    counts = []
    reader = threading.Thread(target=_reader, args=(torch, done, counts, errors))
    reader.start()
    try:
        _run_lane(1, torch, steps, together, errors)
    finally:
        done.set()
        reader.join(timeout=240)
    assert not reader.is_alive()
    assert not errors, errors
    assert counts and counts[0] >= 1
    for (xs, vs), (xp, vp) in zip(alone[1], together[1]):
        assert np.array_equal(xs, xp) and np.array_equal(vs, vp)
