"""Batched and served grids on the GPU: every grid advanced inside a batch (one launch per pass
over all running grids of a precision, optionally replayed from a captured HIP graph) must end
bitwise equal to the same grid advanced alone, whatever else shares the batch and whenever it
was admitted.  Solo runs are themselves parity-checked against the oracle in
test_gpu_parity.py, so equality here carries that parity over to the batched form."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_1410_4194_amd import workloads as WL


@pytest.fixture(scope="module")
def ctu():
    from paper_1410_4194_amd import ctu as _ctu
    return _ctu


def _announce(*parts):
    print("[gpu-test]", *parts, flush=True)
    sys.stdout.flush()


def _solo(ctu, wl, prec, nsteps, t_end=float("inf")):
    g = ctu.Grid.from_workload(wl, prec=prec)
    g.advance(nsteps, t_end)
    info = g.info()
    out = g.get_state()
    g.close()
    return out, info.t, info.steps


def _jobs():
    """Uneven periodic KH grids of both precisions and an outflow shock-cloud grid, each
    with its own step budget."""
    kh = WL.kh_batch(count=7, edges=(16, 24, 32, 40), steps=8)
    jobs = []
    for i, wl in enumerate(kh):
        jobs.append((wl, ctu_prec(i), 3 + (i * 5) % 9))
    jobs.append((WL.shock_cloud(24), 0, 6))
    jobs.append((WL.random_state(20, 12, 9, seed=41, bc=(1,) * 6), 1, 5))
    return jobs


def ctu_prec(i):
    return 0 if i % 3 else 1  # FP64 = 0, FP32 = 1


def _serve(ctu, batch, jobs, run_steps, submit_order=None, stagger=0):
    """Admit jobs as slots free up (optionally only after `stagger` run calls per admission
    wave), run, poll; returns {job index: (state, t)}."""
    grids = [ctu.Grid.from_workload(wl, prec=prec) for wl, prec, _ in jobs]
    order = list(submit_order if submit_order is not None else range(len(jobs)))
    tickets, results = {}, {}
    calls = 0
    while order or tickets:
        if calls % (stagger + 1) == 0:
            while order:
                i = order[0]
                t = batch.submit(grids[i], jobs[i][2])
                if t is None:
                    break
                tickets[t] = order.pop(0)
        batch.run(run_steps)
        calls += 1
        for t in list(tickets):
            state, tnow = batch.poll(t)
            if state in (ctu.TICKET_DONE, ctu.TICKET_FAILED):
                assert state == ctu.TICKET_DONE, (t, state)
                i = tickets.pop(t)
                results[i] = (grids[i].get_state(), tnow, grids[i].info().steps)
        assert calls < 200
    for g in grids:
        g.close()
    return results


@pytest.mark.parametrize("graph", [False, True], ids=["eager", "graph"])
def test_batch_matches_solo(ctu, graph):
    jobs = _jobs()
    _announce("batch vs solo", "graph" if graph else "eager", len(jobs), "jobs")
    solo = [_solo(ctu, wl, prec, n) for wl, prec, n in jobs]
    b = ctu.Batch(max_slots=4, graph=graph)
    res = _serve(ctu, b, jobs, run_steps=2)
    b.close()
    for i, (wl, prec, n) in enumerate(jobs):
        U, t, steps = res[i]
        assert steps == n == solo[i][2], (wl.name, steps, n)
        assert t == solo[i][1]
        assert np.array_equal(U, solo[i][0]), wl.name


def test_batch_long_run_matches_solo_in_order(ctu):
    """A race between the batch's two streams (or between the branches of its captured graph)
    would show as a difference from the same grid advanced alone with every pass in order:
    six Kelvin-Helmholtz grids of edges 48-96 in both precisions, 150 graph-replayed steps
    each, end bitwise equal to those solo runs."""
    kh = WL.kh_batch(count=6, edges=(48, 64, 96), steps=150)
    jobs = [(wl, i % 2, 150) for i, wl in enumerate(kh)]
    _announce("batch long run vs solo in order", len(jobs), "jobs")
    solo = []
    for wl, prec, n in jobs:
        g = ctu.Grid.from_workload(wl, prec=prec, schedule=ctu.SCHEDULE_IN_ORDER)
        g.advance(n)
        info = g.info()
        solo.append((g.get_state(), info.t, info.steps))
        g.close()
    b = ctu.Batch(max_slots=len(jobs), graph=True)
    res = _serve(ctu, b, jobs, run_steps=50)
    b.close()
    for i, (wl, prec, n) in enumerate(jobs):
        U, t, steps = res[i]
        assert steps == n == solo[i][2], (wl.name, steps, n)
        assert t == solo[i][1], wl.name
        assert np.array_equal(U, solo[i][0]), wl.name


def test_graph_replays_match_eager(ctu):
    """The captured step is replayed many times, with eager work and host synchronization
    between replays and recaptures whenever the set of grids changes; every grid, finishing
    at a different replay, must equal the eager batch."""
    jobs = _jobs()
    _announce("graph replays vs eager", len(jobs), "jobs")
    eager = _serve(ctu, ctu.Batch(max_slots=3, graph=False), jobs, run_steps=1, stagger=1)
    graph = _serve(ctu, ctu.Batch(max_slots=3, graph=True), jobs, run_steps=1, stagger=1)
    for i in range(len(jobs)):
        assert np.array_equal(eager[i][0], graph[i][0]), jobs[i][0].name
        assert eager[i][1] == graph[i][1]


def test_alone_equals_in_the_mix(ctu):
    """A request admitted while others are mid-flight (continuous batching) ends the same as
    when it runs alone in a batch."""
    jobs = _jobs()
    probe = len(jobs) - 1
    _announce("alone vs in the mix")
    alone = _serve(ctu, ctu.Batch(max_slots=1), [jobs[probe]], run_steps=3)[0]
    order = [0, 1, 2, probe] + [i for i in range(3, len(jobs) - 1)]
    mixed = _serve(ctu, ctu.Batch(max_slots=5, graph=True), jobs, run_steps=3,
                   submit_order=order, stagger=1)[probe]
    assert np.array_equal(alone[0], mixed[0])
    assert alone[1] == mixed[1] and alone[2] == mixed[2]


def test_batch_end_time_and_budget(ctu):
    """t_end clips the last step (ticket DONE with budget left); a zero budget is DONE at
    once; both equal the solo advance."""
    wl = WL.kelvin_helmholtz(24, 16, 8)
    _announce("batch t_end")
    ref, t_ref, n_ref = _solo(ctu, wl, ctu.FP64, 50, t_end=0.02)
    assert t_ref == 0.02 and n_ref < 50
    g = ctu.Grid.from_workload(wl, prec=ctu.FP64)
    g0 = ctu.Grid.from_workload(wl, prec=ctu.FP32)
    b = ctu.Batch(max_slots=2)
    t = b.submit(g, 50, 0.02)
    t0 = b.submit(g0, 0)
    assert b.poll(t0)[0] == ctu.TICKET_DONE
    for _ in range(60):
        b.run(1)
        state, tnow = b.poll(t)
        if state != ctu.TICKET_RUNNING:
            break
    assert state == ctu.TICKET_DONE and tnow == 0.02
    assert np.array_equal(g.get_state(), ref)
    assert g0.info().steps == 0


def test_failed_ticket_leaves_others_intact(ctu):
    """A grid whose state turns non-physical is FAILED and stops; its neighbours in the batch
    are unaffected."""
    good = WL.kelvin_helmholtz(16, 16, 16)
    bad = WL.random_state(16, 8, 8, seed=23)
    _announce("failed ticket")
    ref, _, _ = _solo(ctu, good, ctu.FP64, 6)
    gb = ctu.Grid.from_workload(bad, prec=ctu.FP64)
    U = gb.get_state()
    U[0, 3, 4, 5] = np.nan
    gb.set_state(U)
    gg = ctu.Grid.from_workload(good, prec=ctu.FP64)
    b = ctu.Batch(max_slots=2, graph=True)
    tb = b.submit(gb, 6)
    tg = b.submit(gg, 6)
    b.run(6)
    assert b.poll(tb)[0] == ctu.TICKET_FAILED
    assert b.poll(tg)[0] == ctu.TICKET_DONE
    assert np.array_equal(gg.get_state(), ref)
    status, flags, _ = gb.check()
    assert status == ctu.ENONPHYS and flags & ctu.FLAG_NONFINITE


def test_submitted_grid_is_locked(ctu):
    wl = WL.kelvin_helmholtz(16, 16, 16)
    g = ctu.Grid.from_workload(wl, prec=ctu.FP64)
    b = ctu.Batch(max_slots=1)
    t = b.submit(g, 2)
    assert b.submit(ctu.Grid.from_workload(wl), 2) is None  # no free slot
    for call in (lambda: g.step(1e-3), lambda: g.advance(1), g.get_state, g.compute_dt):
        with pytest.raises(ctu.CtuError) as ei:
            call()
        assert ei.value.status == ctu.EINVAL
    b.run(2)
    assert b.poll(t)[0] == ctu.TICKET_DONE
    assert g.info().steps == 2
    assert b.poll(t)[0] == ctu.TICKET_UNKNOWN



def test_batch_mixed_gas_classes(ctu):
    """Grids of different gamma (each gas class is its own kernel group) and both precisions
    in one batch, each equal to its solo run."""
    jobs = [(WL.random_state(14, 11, 9, seed=61, gamma=1.3), 0, 4),
            (WL.random_state(12, 10, 13, seed=62, gamma=5.0 / 3.0), 1, 5),
            (WL.random_state(9, 16, 10, seed=63, gamma=1.4, bc=(1,) * 6), 0, 3),
            (WL.random_state(10, 9, 12, seed=64, gamma=9.0 / 7.0), 1, 4),
            (WL.random_state(11, 12, 8, seed=65, gamma=5.0 / 3.0), 0, 6)]
    _announce("mixed gas classes")
    solo = [_solo(ctu, wl, prec, n) for wl, prec, n in jobs]
    res = _serve(ctu, ctu.Batch(max_slots=5, graph=True), jobs, run_steps=2)
    for i, (wl, prec, n) in enumerate(jobs):
        assert res[i][2] == n and np.array_equal(res[i][0], solo[i][0]), wl.name