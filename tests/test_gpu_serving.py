"""Serving runtime (igamg_server_*): continuous batching of heterogeneous
requests, admission by memory footprint, and results that do not depend on
the other requests in flight.

Tolerances: a request's arithmetic is the same alone and in a mix, and every
sum on the path has a fixed order, so float64 results are bitwise equal.
Float32 requests (switched off, see below) would be held to the same
residual bar and 1e-6 relative.
"""
import numpy as np
import pytest

import workloads
from paper_1902_01818_amd import serve
from tests.gpu_common import max_abs_rel, oracle_iterate, oracle_problem, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _specs():
    # small heterogeneous requests: layouts, degrees and element counts differ
    out = []
    for i, (a, b, p, n0) in enumerate([(2, 2, 2, 16), (3, 2, 3, 16), (2, 3, 4, 32), (4, 4, 2, 16),
                                       (3, 3, 5, 16), (2, 2, 6, 32)]):
        out.append(dict(counts=(a, b), p=p, n0=n0, n1=3 * n0 // 2, geom_seed=100 + i,
                        rhs_seed=200 + i))
    return out


def _run(problems, slots, budget=4 << 30, rate=None):
    from paper_1902_01818_amd import igamg
    srv = igamg.Server(slots=slots, memory_budget=budget)
    try:
        recs, summ = serve.run(srv, problems, rate=rate)
        st = srv.status()
    finally:
        srv.close()
    return recs, summ, st


FP32_OFF = ("float32 requests are switched off in the serving runtime: their first run "
            "aborted the process without a message and the cause is not identified")


@pytest.mark.parametrize("precision,outer", [
    ("fp64", "pcg"),
    pytest.param("fp32", "fcg", marks=pytest.mark.skip(reason=FP32_OFF))])
def test_alone_equals_mix(precision, outer):
    problems = serve.prepare(_specs(), precision, outer)
    alone = []
    for pb in problems:
        recs, _, _ = _run([pb], slots=1)
        alone.append(recs[0])
    mix, summ, _ = _run(problems, slots=4)
    assert summ["completed"] == len(problems) == summ["converged"]
    for (ua, ia), (um, im) in zip(alone, mix):
        assert ia["status"] == 0 and im["status"] == 0
        assert ia["true_rel_residual"] <= 1e-8 and im["true_rel_residual"] <= 1e-8
        assert im["fallback_allocations"] == 0
        if precision == "fp64":
            assert np.array_equal(np.asarray(um), np.asarray(ua))
            assert ia["iterations"] == im["iterations"]
        else:
            assert rel_err(um, ua) < 1e-6
            assert abs(ia["iterations"] - im["iterations"]) <= 1


def test_serving_matches_oracle():
    spec = _specs()[1]
    pb = serve.prepare([spec], "fp64", "pcg")[0]
    recs, _, _ = _run([pb], slots=1)
    u, info = recs[0]
    prob = workloads.request_problem(spec)
    ob = oracle_problem(prob)
    uo, its, _, iterates = ob.pcg(pb["rhs"])
    kg = info["iterations"]
    assert abs(kg - its) <= 1
    ui = oracle_iterate(ob, pb["rhs"], kg, its, iterates)
    assert rel_err(u, ui) < 1e-10
    assert max_abs_rel(u, ui) < 1e-10


def test_admission_by_footprint():
    problems = serve.prepare(_specs(), "fp64", "pcg")
    # learn the footprints, then give the server room for the largest request only
    recs, _, _ = _run(problems, slots=4)
    fps = [r[1]["footprint"] for r in recs]
    budget = int(max(fps) * 1.1)
    recs, summ, st = _run(problems, slots=4, budget=budget)
    assert summ["completed"] == len(problems) == summ["converged"]
    assert st["peak_reserved"] <= budget
    # with room for about one request at a time, later requests waited in the queue
    assert summ["mean_queue_s"] > 0


def test_request_larger_than_budget_is_rejected():
    problems = serve.prepare(_specs()[:2], "fp64", "pcg")
    recs, _, _ = _run(problems, slots=2)
    small = min(r[1]["footprint"] for r in recs)
    big = max(r[1]["footprint"] for r in recs)
    if small == big:
        pytest.skip("requests of equal footprint")
    recs, summ, _ = _run(problems, slots=2, budget=int((small + big) / 2))
    codes = sorted(r[1]["status"] for r in recs)
    assert codes == [-3, 0]   # IGAMG_ENOMEM for the request that can never fit


def test_float32_requests_rejected_at_submission():
    """Float32 requests are refused before they are queued (the server runs
    float64 requests only); no solve is started."""
    from paper_1902_01818_amd import igamg
    pb = serve.prepare(_specs()[:1], "fp32", "fcg")[0]
    srv = igamg.Server(slots=1, memory_budget=1 << 30)
    try:
        with pytest.raises(igamg.IgamgError) as e:
            srv.submit(pb["corners"], pb["elems"], pb["p"], pb["rhs"], sigma=pb["sigma"],
                       **pb["opts"])
        assert e.value.code == igamg.EUNSUPPORTED
        assert srv.status()["queued"] == 0
    finally:
        srv.close()
