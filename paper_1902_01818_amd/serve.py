"""Request-stream driver of the serving runtime (igamg_server_*).

A seeded stream of heterogeneous 2D SIPG solve requests (patch layouts,
degrees and element counts drawn per request) arrives with exponential
inter-arrival times; every request is submitted to the native server at its
arrival time and its latency is measured from submission to result on the
server's clock (setup included).  All scheduling, admission and solving
happen in the library; this module only paces submissions and collects the
records.

    python -m paper_1902_01818_amd.serve [--requests 2000] [--slots 4]
        [--budget-gib 200] [--load 0.7] [--calibrate 64]
"""
import argparse
import json
import os
import sys
import threading
import time

import numpy as np

_ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if _ROOT not in sys.path:
    sys.path.insert(0, _ROOT)

from paper_1902_01818_amd import igamg  # noqa: E402


def prepare(reqs, precision="fp64", outer="pcg"):
    """Problem arrays, sizes and right-hand sides of a list of request specs
    (generated before the stream starts, so that pacing is not delayed)."""
    import workloads
    out = []
    for r in reqs:
        pb = workloads.request_problem(r)
        opts = dict(conforming=False, smoother=pb["smoother"], tau=pb["tau"], delta=pb["delta"],
                    precision=precision, outer=outer)
        n, _ = igamg.problem_size(pb["corners"], pb["elems"], pb["p"], **opts)
        rhs = workloads.normal_rhs(n, pb["rhs"][1])
        out.append(dict(corners=pb["corners"], elems=pb["elems"], p=pb["p"], sigma=pb["sigma"],
                        opts=opts, rhs=rhs, n=n))
    return out


def run(server, problems, rate=None, tol=1e-8, maxit=200, seed=0, progress=0):
    """Submit `problems` (from prepare) at Poisson arrivals of `rate` per second
    (None: all at once) and wait for all.  Returns per-request records and the
    stream's summary."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, len(problems)) if rate else np.zeros(len(problems))
    ids = [None] * len(problems)
    err = []

    def submitter():
        t = time.perf_counter()
        for i, pb in enumerate(problems):
            t += gaps[i]
            dt = t - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            try:
                ids[i] = server.submit(pb["corners"], pb["elems"], pb["p"], pb["rhs"],
                                       sigma=pb["sigma"], tol=tol, maxit=maxit, **pb["opts"])
            except Exception as e:  # input errors are reported per request
                err.append((i, str(e)))

    th = threading.Thread(target=submitter)
    th.start()
    th.join()
    recs = []
    for i, rid in enumerate(ids):
        if rid is None:
            continue
        u, info = server.wait(rid)
        info["index"] = i
        info["latency"] = info["t_done"] - info["t_submit"]
        recs.append((u, info))
        if progress and len(recs) % progress == 0:
            print("serving: %d/%d requests done" % (len(recs), len(problems)), file=sys.stderr,
                  flush=True)
    infos = [r[1] for r in recs]
    ok = [i for i in infos if i["status"] == 0 and i["true_rel_residual"] <= tol * 1.05]
    lat = np.array([i["latency"] for i in infos]) if infos else np.zeros(1)
    span = (max(i["t_done"] for i in infos) - min(i["t_submit"] for i in infos)) if infos else 0.0
    summary = dict(requests=len(problems), completed=len(infos), converged=len(ok),
                   submit_errors=len(err),
                   solves_per_s=len(infos) / span if span > 0 else None,
                   p50_latency_s=float(np.percentile(lat, 50)),
                   p99_latency_s=float(np.percentile(lat, 99)),
                   mean_setup_s=float(np.mean([i["t_ready"] - i["t_admit"] for i in infos])) if infos else None,
                   mean_queue_s=float(np.mean([i["t_admit"] - i["t_submit"] for i in infos])) if infos else None,
                   fallback_allocations=int(sum(i["fallback_allocations"] for i in infos)),
                   dofs_total=int(sum(i["n_dofs"] for i in infos)))
    return recs, summary


def serve_benchmark(n_requests=2000, slots=4, budget_gib=200.0, load=0.7, calibrate=64,
                    master_seed=5000, precision="fp64", outer="pcg"):
    """The serving workload: a calibration burst measures saturated throughput,
    then the stream arrives at `load` times that rate."""
    import workloads
    reqs = workloads.serving_requests(n_requests, master_seed)
    problems = prepare(reqs, precision, outer)
    srv = igamg.Server(slots=slots, memory_budget=int(budget_gib * (1 << 30)))
    try:
        # saturated throughput of an evenly spaced sample of the whole stream
        stride = max(1, len(problems) // max(1, calibrate))
        _, cal = run(srv, problems[::stride][:calibrate], rate=None, progress=16)
        rate = load * cal["solves_per_s"]
        _, summ = run(srv, problems, rate=rate, seed=master_seed, progress=16)
        st = srv.status()
    finally:
        srv.close()
    summ.update(arrival_rate_per_s=rate, saturated_solves_per_s=cal["solves_per_s"],
                load=load, slots=slots, budget_gib=budget_gib,
                peak_reserved_gib=st["peak_reserved"] / (1 << 30), precision=precision,
                outer=outer)
    return summ


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--budget-gib", type=float, default=200.0)
    ap.add_argument("--load", type=float, default=0.7)
    ap.add_argument("--calibrate", type=int, default=64)
    ap.add_argument("--precision", default="fp64")
    a = ap.parse_args()
    outer = "fcg" if a.precision == "fp32" else "pcg"
    print(json.dumps(serve_benchmark(a.requests, a.slots, a.budget_gib, a.load, a.calibrate,
                                     precision=a.precision, outer=outer)))


if __name__ == "__main__":
    main()
