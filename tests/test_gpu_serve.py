"""Serving loop on the GPU: Poisson-arriving shock-cloud requests of different sizes, admitted
by HBM footprint into a continuous batch, in arrival order or least estimated work first.
Every answer must equal the same request solved alone (bitwise: each grid's arithmetic does
not depend on what shares the batch), the HBM budget must hold at all times, and requests
must actually overlap."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_1410_4194_amd import workloads as WL


def _announce(*parts):
    print("[gpu-test]", *parts, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("policy", ["fifo", "sjf"])
@pytest.mark.parametrize("prec", [1, 0], ids=["fp32", "fp64"])
def test_served_answers_equal_solo(prec, policy):
    from paper_1410_4194_amd import ctu, serve as S
    reqs = WL.shock_cloud_requests(10, rate=200.0, sizes=(16, 24, 32), t_cc_factor=0.05)
    requests = [S.Request(q["rid"], q["arrival"], WL.request_workload(q), q["t_end"], prec,
                          cost=WL.estimated_steps(q) * q["n"] ** 3)
                for q in reqs]
    foot = [S.footprint(r) for r in requests]
    budget = int(2.5 * max(foot))  # admission is limited by memory, not only by slots
    _announce("serve", len(requests), "requests, budget", budget, "bytes, prec", prec,
              "policy", policy)
    stats = S.serve(requests, hbm_budget=budget, max_slots=6, steps_per_round=2,
                    keep_states=True, policy=policy)
    assert len(stats.results) == len(requests)
    assert stats.max_resident_bytes <= budget
    assert stats.max_concurrent >= 2
    for req, res in zip(requests, stats.results):
        assert res.rid == req.rid and res.steps > 0
        assert abs(res.t - req.t_end) <= 1e-14 * req.t_end
        # the same request, with the same configuration (the batch tile shapes), alone
        g = ctu.Grid.from_workload(req.workload, prec=prec, batch=True)
        g.advance(res.steps + 3, req.t_end)
        info = g.info()
        assert info.steps == res.steps and info.t == res.t
        assert np.array_equal(g.get_state(), res.state), req.rid
        g.close()
    s = stats.summary()
    _announce("p50", s["p50_s"], "p99", s["p99_s"], "max concurrent", s["max_concurrent"])
    assert s["p99_s"] >= s["p50_s"] > 0
