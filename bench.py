"""Benchmark: solves/s of the hybrid-smoother multigrid PCG solver to relative
residual 1e-8 on one MI355X, with the roofline position of the dominant
kernel and the FP64 CPU oracle timed on the host beside it.

Workload (default): 2D SIPG on the unit square split into 4x4 bilinear
patches (corners perturbed by up to 10% of the patch width, seed 1902),
checkerboard 64/96 elements per direction (non-matching interfaces),
degree 4, penalty 5 p^2/h, V(1,1) cycle with the hybrid smoother
(forward Gauss-Seidel + SCMS / SCMS + backward Gauss-Seidel, damping 0.25,
scaling 0.1), float64 PCG, N(0,1) right-hand side (seed 2002), 115,652
unknowns.  Levels: uniform halving down to 8/12 elements per patch (4 levels,
dense direct solve of the 2,940-unknown coarsest level on the GPU);
--coarse-min 2 halves down to 2/3 elements (6 levels).  One step = one
complete solve; the right-hand side is resident in HBM before the timed
region starts.  Also reported: the float32-cycle solve (float64 flexible CG)
and a serving sample (p50/p99 latency).

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X peaks: HBM GB/s; vector and MFMA TFLOP/s (dense MFMA: f64 78.6,
# f32 157.3, bf16 2500)
PEAK = {"hbm": 8000.0, "fp64": 78.6, "fp32": 157.3}
MFMA_PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}


KERNEL_OF_FAMILY = {"gauss_seidel": "gs2d_wave_kernel", "vol_apply": "vol2d_kernel",
                    "scms": "fd2m_kernel", "iface_apply": "iface_kernel",
                    "stencil_apply": "sp2d_kernel"}


def source_hash(family="gauss_seidel"):
    """Hash of the device source of the family's kernel (its definition in
    kernels.hip): counter-based traffic figures are valid only for the kernel
    they were measured on."""
    import hashlib
    src = open(os.path.join(ROOT, "paper_1902_01818_amd", "csrc", "kernels.hip")).read()
    name = KERNEL_OF_FAMILY[family]
    i = src.index("void %s(" % name)
    j = src.index("\n}\n", i)
    return hashlib.sha256(src[i:j].encode()).hexdigest()[:16]


def cpu_baseline(cfg, f, its_gpu, budget_s=15.0):
    """Oracle (plain FP64 CPU reference) on the same workload: setup excluded
    (as on the GPU), full PCG solves repeated until budget_s of CPU work."""
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = 1
    pb = oracle.setup(cfg["corners"], cfg["elems"], cfg["p"], sigma=cfg["sigma"],
                      conforming=cfg["conforming"], smoother=cfg["smoother"], tau=cfg["tau"],
                      delta=cfg["delta"])
    n = 0
    t0 = time.perf_counter()
    its = None
    while True:
        _, its, _, _ = pb.pcg(f)
        n += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return dict(value=n / dt, unit="solves/s", cores=int(threads), kind="oracle",
                sample="%d full PCG solve(s) of the benchmark problem (%d iterations each, "
                       "setup excluded), %.1f s" % (n, its, dt),
                iterations=its)


def c4_leg(igamg, torch, workloads, nrhs=64, precision="fp32", steps=2, outer=None):
    """64 right-hand sides of the p = 6, 256-element workload solved together
    (float32 cycle, optionally with bfloat16 SCMS contractions, inside float64
    flexible CG; or float64 PCG), with the matrix-core utilisation of the
    finest level's SCMS application measured in one more, event-timed solve."""
    cfg = workloads.config("c4")
    if outer is None:
        outer = "pcg" if precision == "fp64" else "fcg"
    t0 = time.perf_counter()
    sv = igamg.Solver(cfg["corners"], cfg["elems"], cfg["p"], cfg["sigma"],
                      conforming=cfg["conforming"], smoother=cfg["smoother"], tau=cfg["tau"],
                      delta=cfg["delta"], precision=precision, outer=outer, max_rhs=nrhs)
    setup_s = time.perf_counter() - t0
    n = sv.n_dofs
    F = torch.from_numpy(np.stack([workloads.normal_rhs(n, 4000 + j) for j in range(nrhs)])).cuda()
    U = torch.zeros_like(F)
    sv.solve(F, U, tol=1e-8, maxit=200)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        _, info = sv.solve(F, U, tol=1e-8, maxit=200)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    its = [i["iterations"] for i in info]
    out = dict(workload="C2 geometry, p=6, 256 elements/patch, %d N(0,1) right-hand sides" % nrhs,
               dofs=n, precision=precision, outer=outer, solves_per_s=nrhs / dt,
               ms_per_batch=dt * 1e3, setup_s=setup_s, memory_gib=sv.memory() / (1 << 30),
               iterations_max=max(its), iterations_min=min(its),
               max_true_rel_residual=max(i["true_rel_residual"] for i in info),
               all_converged=all(i["converged"] for i in info))
    top = sv.n_levels - 1
    key = "scms/%d" % top
    sv.set_timing(key)
    sv.solve(F, U, tol=1e-8, maxit=200)
    torch.cuda.synchronize()
    st = sv.kernel_stats(reset=True)
    sv.set_timing(None)
    if st.get(key, {}).get("launches"):
        avg = st[key]["ms"] / 1e3 / st[key]["launches"]
        _, fl = sv.kernel_model("scms", top, nrhs)
        ach = fl / avg / 1e12
        peak = MFMA_PEAK["bf16" if precision == "bf16" else precision]
        out["scms_mfma"] = dict(kernel=key, bound="mfma", achieved=ach, peak=peak,
                                unit="TFLOP/s", frac=ach / peak, avg_application_us=avg * 1e6,
                                model_flops_per_application=fl)
    sv.close()
    return out


def c1_leg(igamg, torch, workloads, steps=20, batch=1000):
    """The conforming 2x2 workload (p = 2, 16 elements, SCMS V(1,1), float64
    PCG): single-solve and V-cycle rates, a batch of `batch` right-hand sides
    solved together, and the L2 error of the manufactured solution on a
    ladder of element counts with the observed order."""
    cfg = workloads.config("c1")
    opts = dict(conforming=cfg["conforming"], smoother=cfg["smoother"], tau=cfg["tau"],
                delta=cfg["delta"])
    sv = igamg.Solver(cfg["corners"], cfg["elems"], cfg["p"], cfg["sigma"], **opts)
    f = sv.load_manufactured()
    u, info = sv.solve(f, tol=1e-8, maxit=200)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        u, info = sv.solve(f, tol=1e-8, maxit=200)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    v = torch.zeros_like(f)
    sv.vcycle(f, v)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10 * steps):
        sv.vcycle(f, v)
    torch.cuda.synchronize()
    dv = (time.perf_counter() - t0) / (10 * steps)
    out = dict(workload="conforming 2x2 identity patches, p=2, 16 elements, SCMS V(1,1), "
                        "manufactured", dofs=sv.n_dofs, levels=sv.n_levels,
               iterations=info[0]["iterations"], solves_per_s=1.0 / dt, vcycles_per_s=1.0 / dv,
               l2_error=sv.l2_error(u))
    sv.close()
    # many instances of the problem at once: one right-hand side each
    sb = igamg.Solver(cfg["corners"], cfg["elems"], cfg["p"], cfg["sigma"], max_rhs=batch, **opts)
    F = torch.from_numpy(np.stack([workloads.normal_rhs(sb.n_dofs, 6000 + j)
                                   for j in range(batch)])).cuda()
    U, infos = sb.solve(F, tol=1e-8, maxit=200)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    U, infos = sb.solve(F, tol=1e-8, maxit=200)
    torch.cuda.synchronize()
    out["batched"] = dict(rhs=batch, solves_per_s=batch / (time.perf_counter() - t0),
                          iterations_max=max(i["iterations"] for i in infos),
                          all_converged=all(i["converged"] for i in infos))
    sb.close()
    # L2 error ladder (order p+1 = 3 expected)
    ladder = []
    for ne in (4, 8, 16, 32, 64):
        el = np.full((4, 2), ne)
        s2 = igamg.Solver(cfg["corners"], el, cfg["p"], cfg["sigma"], **opts)
        g = s2.load_manufactured()
        w, _ = s2.solve(g, tol=1e-12, maxit=200)
        ladder.append((ne, s2.l2_error(w)))
        s2.close()
    out["l2_ladder"] = [dict(elements=ne, l2_error=e,
                             order=(None if i == 0 else
                                    float(np.log2(ladder[i - 1][1] / e))))
                        for i, (ne, e) in enumerate(ladder)]
    return out


def c3_leg(igamg, torch, workloads, precision="fp32", steps=2, operator_apply="auto"):
    """The 3D workload at full size (2x2x2 trilinear patches, 48/64 elements,
    p = 3, 1.65 M unknowns, manufactured right-hand side), hybrid cycle in
    the given arithmetic inside float64 flexible CG (float64: PCG), plus the
    time per kernel family of one more, event-timed solve."""
    cfg = workloads.config("c3")
    outer = "pcg" if precision == "fp64" else cfg["outer"]
    t0 = time.perf_counter()
    sv = igamg.Solver(cfg["corners"], cfg["elems"], cfg["p"], cfg["sigma"],
                      conforming=cfg["conforming"], smoother=cfg["smoother"], tau=cfg["tau"],
                      delta=cfg["delta"], precision=precision, outer=outer,
                      operator_apply=operator_apply)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    f = sv.load_manufactured()
    u, info = sv.solve(f, tol=1e-8, maxit=200)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        u, info = sv.solve(f, tol=1e-8, maxit=200)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    out = dict(workload="3D SIPG, 2x2x2 trilinear patches, 48/64 elements, p=3, manufactured",
               dofs=sv.n_dofs, levels=sv.n_levels, precision=precision, outer=outer,
               operator_apply=operator_apply,
               solves_per_s=1.0 / dt, ms_per_solve=dt * 1e3, setup_s=setup_s,
               memory_gib=sv.memory() / (1 << 30), iterations=info[0]["iterations"],
               true_rel_residual=info[0]["true_rel_residual"], converged=info[0]["converged"])
    sv.set_timing("")
    sv.solve(f, tol=1e-8, maxit=200)
    torch.cuda.synchronize()
    st = sv.kernel_stats(reset=True)
    sv.set_timing(None)
    fam = {}
    for k, v in st.items():
        name = k.split("/")[0]
        fam[name] = fam.get(name, 0.0) + v["ms"]
    out["ms_per_family_timed_solve"] = {k: round(v, 3) for k, v in sorted(fam.items())}
    # the finest level's operator kernels: average launch and model rate
    top = sv.n_levels - 1
    key = "scms/%d" % top
    if st.get(key, {}).get("launches"):
        avg = st[key]["ms"] / 1e3 / st[key]["launches"]
        _, fl = sv.kernel_model("scms", top, 1)
        peak = MFMA_PEAK["bf16" if precision == "bf16" else precision]
        out["scms_mfma"] = dict(kernel=key, bound="mfma", achieved=fl / avg / 1e12, peak=peak,
                                unit="TFLOP/s", frac=fl / avg / 1e12 / peak,
                                avg_application_us=avg * 1e6, model_flops_per_application=fl)
    for famname in ("vol_apply", "stencil_apply"):
        key = "%s/%d" % (famname, top)
        if st.get(key, {}).get("launches"):
            avg = st[key]["ms"] / 1e3 / st[key]["launches"]
            b, fl = sv.kernel_model(famname, top, 1)
            out["finest_" + famname] = dict(avg_us=avg * 1e6, model_gb_s=b / avg / 1e9,
                                            model_tflop_s=fl / avg / 1e12)
    sv.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the float32-cycle run")
    ap.add_argument("--serve-budget-gib", type=float, default=64.0,
                    help="device memory the serving runtime admits requests into")
    ap.add_argument("--serve-requests", type=int, default=96,
                    help="requests of the serving sample (0 = skip)")
    ap.add_argument("--no-c4", action="store_true", help="skip the 64-column p = 6 workload")
    ap.add_argument("--c4-only", action="store_true",
                    help="diagnostic: run only the 64-column p = 6 legs (float32 cycle, bf16 "
                         "SCMS) and print their results (not the benchmark line)")
    ap.add_argument("--c1-only", action="store_true",
                    help="diagnostic: run only the conforming 2x2 workload (rates, a batch of "
                         "1000 right-hand sides, L2 error ladder) and print its results")
    ap.add_argument("--c3-only", action="store_true",
                    help="diagnostic: run only the full-size 3D workload (float32 and float64 "
                         "cycles) and print its results (not the benchmark line)")
    ap.add_argument("--coarse-min", type=int, default=8,
                    help="halving stops before an element count falls below this: 8 puts the "
                         "direct solve on the 8/12-element level (2,940 unknowns, 4 levels); "
                         "2 halves down to 2/3 elements (6 levels)")
    ap.add_argument("--family", default=None, help="kernel family for the roofline entry")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after the timed region, copy MIB MiB device to device (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads
    from paper_1902_01818_amd import igamg

    if args.c1_only:
        print(json.dumps({"c1": c1_leg(igamg, torch, workloads)}))
        return

    if args.c3_only:
        out = {"c3": c3_leg(igamg, torch, workloads, precision="fp32")}
        print("bench: 3D workload timed (float32 cycle)", file=sys.stderr, flush=True)
        out["c3_fp64"] = c3_leg(igamg, torch, workloads, precision="fp64")
        print("bench: 3D workload timed (float64 cycle)", file=sys.stderr, flush=True)
        out["c3_sumfact"] = c3_leg(igamg, torch, workloads, precision="fp32",
                                   operator_apply="sumfact")
        print("bench: 3D workload timed (matrix-free operator)", file=sys.stderr, flush=True)
        out["c3_bf16_scms"] = c3_leg(igamg, torch, workloads, precision="bf16")
        out["mixed_speedup"] = {k: out[k]["solves_per_s"] / out["c3_fp64"]["solves_per_s"]
                                for k in ("c3", "c3_bf16_scms")}
        print(json.dumps(out))
        return

    if args.c4_only:
        out = {"c4": c4_leg(igamg, torch, workloads, nrhs=64, precision="fp32", steps=1)}
        print("bench: 64-column p = 6 batch timed (float32 cycle)", file=sys.stderr, flush=True)
        out["c4_bf16_scms"] = c4_leg(igamg, torch, workloads, nrhs=64, precision="bf16", steps=1)
        print("bench: 64-column p = 6 batch timed (bf16 SCMS)", file=sys.stderr, flush=True)
        out["c4_fp64"] = c4_leg(igamg, torch, workloads, nrhs=64, precision="fp64", steps=1)
        print(json.dumps(out))
        return

    cfg = workloads.config("c2")
    sv = igamg.Solver(cfg["corners"], cfg["elems"], cfg["p"], cfg["sigma"],
                      conforming=cfg["conforming"], smoother=cfg["smoother"], tau=cfg["tau"],
                      delta=cfg["delta"], timing=False, coarse_min=args.coarse_min)
    N = sv.n_dofs
    f_host = workloads.normal_rhs(N, cfg["rhs"][1])
    f = torch.from_numpy(f_host).cuda()
    u = torch.zeros_like(f)
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        sv.solve(f, u, tol=1e-8, maxit=200)
    torch.cuda.synchronize()

    # dominant kernel on the finest level: the family with the most event time
    # in one untimed instrumented solve
    top = sv.n_levels - 1
    family = args.family
    if family is None:
        sv.set_timing("")
        sv.solve(f, u, tol=1e-8, maxit=200)
        st = sv.kernel_stats(reset=True)
        fams = {}
        for key, v in st.items():
            fam = key.split("/")[0]
            fams[fam] = fams.get(fam, 0.0) + v["ms"]
        modelled = [k for k in KERNEL_OF_FAMILY if k in fams]
        family = max(modelled, key=lambda k: fams[k])
    # timed region: only the dominant family on the finest level is event-timed
    sv.set_timing("%s/%d" % (family, top))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for _ in range(args.steps):
        _, info = sv.solve(f, u, tol=1e-8, maxit=200)
        infos.append(info[0])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = sv.kernel_stats(reset=True)
    sv.set_timing(None)
    print("bench: float64 solves timed (%.1f ms/solve)" % (dt / args.steps * 1e3), file=sys.stderr,
          flush=True)
    key = "%s/%d" % (family, top)
    launches = st[key]["launches"]
    avg_s = st[key]["ms"] / 1e3 / max(launches, 1)
    mbytes, mflops = sv.kernel_model(family, top, 1)
    if family == "vol_apply":
        achieved = mflops / avg_s / 1e12
        roof = dict(bound="alu", achieved=achieved, peak=PEAK["fp64"], unit="TFLOP/s")
    elif family == "scms":
        achieved = mflops / avg_s / 1e12
        roof = dict(bound="mfma", achieved=achieved, peak=MFMA_PEAK["fp64"], unit="TFLOP/s")
    else:
        achieved = mbytes / avg_s / 1e9
        roof = dict(bound="hbm", achieved=achieved, peak=PEAK["hbm"], unit="GB/s")
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = None
    roof["kernel"] = key
    roof["avg_launch_us"] = avg_s * 1e6
    roof["launches"] = launches
    roof["model_bytes_per_launch"] = mbytes
    roof["model_flops_per_launch"] = mflops

    # every modelled kernel family of the finest level (and the coarse solve)
    # in one more, event-timed solve: mean launch time and achieved rate
    sv.set_timing("")
    sv.solve(f, u, tol=1e-8, maxit=200)
    torch.cuda.synchronize()
    st_all = sv.kernel_stats(reset=True)
    sv.set_timing(None)
    kernels = {}
    for fam in ("gauss_seidel", "stencil_apply", "vol_apply", "iface_apply", "scms", "pieces",
                "restrict", "prolong", "coarse"):
        k = "%s/%d" % (fam, 0 if fam == "coarse" else top)
        if not st_all.get(k, {}).get("launches"):
            continue
        t = st_all[k]["ms"] / 1e3 / st_all[k]["launches"]
        b, fl = sv.kernel_model(fam, top, 1)
        ent = {"avg_us": t * 1e6, "model_bytes": b, "model_flops": fl,
               "gb_s": b / t / 1e9, "frac_hbm": b / t / 1e9 / PEAK["hbm"]}
        if fam == "scms":
            ent["tflop_s"] = fl / t / 1e12
            ent["frac_mfma_fp64"] = ent["tflop_s"] / MFMA_PEAK["fp64"]
        kernels[fam] = ent

    its = infos[-1]["iterations"]
    ok = all(i["converged"] and i["true_rel_residual"] <= 1e-8 * 1.01 for i in infos)
    value = args.steps / dt
    line = {
        "metric": "solves/s to rel.res 1e-8 (mixed vs FP64 MG), p50/p99 latency, HBM GB/s",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "2D SIPG, 4x4 bilinear patches (10%% seeded perturbation), "
                               "checkerboard 64/96 elements, p=4, sigma=5, hybrid V(1,1) over "
                               "%d levels (dense direct solve on the coarsest), FP64 PCG to 1e-8"
                               % sv.n_levels,
                   "dofs": N, "levels": sv.n_levels, "coarse_min": args.coarse_min,
                   "iterations": its,
                   "vcycles_per_s": value * (its + 1),
                   "true_rel_residual": infos[-1]["true_rel_residual"], "all_converged": ok},
        "roofline": roof,
        "kernels_finest": kernels,
    }
    # mixed precision: float32 cycle inside float64 flexible CG, same workload,
    # same float64 stopping test; error reported against the float64 GPU solve
    if not args.no_mixed:
        u64 = u.clone()
        sm = igamg.Solver(cfg["corners"], cfg["elems"], cfg["p"], cfg["sigma"],
                          conforming=cfg["conforming"], smoother=cfg["smoother"], tau=cfg["tau"],
                          delta=cfg["delta"], precision="fp32", outer="fcg",
                          coarse_min=args.coarse_min)
        um = torch.zeros_like(f)
        for _ in range(args.warmup):
            sm.solve(f, um, tol=1e-8, maxit=200)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        minfo = []
        for _ in range(args.steps):
            _, info = sm.solve(f, um, tol=1e-8, maxit=200)
            minfo.append(info[0])
        torch.cuda.synchronize()
        dtm = time.perf_counter() - t0
        line["mixed"] = {
            "cycle_dtype": "f32", "outer_dtype": "f64", "outer": "flexible CG",
            "value": args.steps / dtm, "unit": "solves/s", "ms_per_step": dtm / args.steps * 1e3,
            "speedup_vs_fp64": (args.steps / dtm) / value,
            "iterations": minfo[-1]["iterations"],
            "true_rel_residual": minfo[-1]["true_rel_residual"],
            "all_converged": all(i["converged"] and i["true_rel_residual"] <= 1e-8 * 1.01
                                 for i in minfo),
            "rel_error_vs_fp64_solution": float(torch.linalg.norm(um - u64) / torch.linalg.norm(u64)),
        }
        sm.close()
        print("bench: float32-cycle solves timed", file=sys.stderr, flush=True)
    # serving: a seeded sample of the heterogeneous request stream arrives at
    # Poisson times (rate = load x the saturated rate of a calibration burst);
    # latency = submission to result, setup included
    if args.serve_requests > 0:
        from paper_1902_01818_amd import serve
        line["serving"] = serve.serve_benchmark(
            n_requests=args.serve_requests, slots=4, budget_gib=args.serve_budget_gib, load=0.7,
            calibrate=min(max(32, args.serve_requests // 16), args.serve_requests))
    # batched right-hand sides (p = 6, 256 elements per patch, 64 columns)
    if not args.no_c4:
        line["c4"] = c4_leg(igamg, torch, workloads, nrhs=64, precision="fp32", steps=1)
        print("bench: 64-column p = 6 batch timed (float32 cycle)", file=sys.stderr, flush=True)
        line["c4_bf16_scms"] = c4_leg(igamg, torch, workloads, nrhs=64, precision="bf16", steps=1)
        print("bench: 64-column p = 6 batch timed (bf16 SCMS)", file=sys.stderr, flush=True)
        line["c4_refinement"] = c4_leg(igamg, torch, workloads, nrhs=64, precision="fp32",
                                       steps=1, outer="ir")
        print("bench: 64-column p = 6 batch timed (float64 iterative refinement)", file=sys.stderr,
              flush=True)
        line["c4_fp64"] = c4_leg(igamg, torch, workloads, nrhs=64, precision="fp64", steps=1)
        line["c4_fp64"]["mixed_speedup"] = {
            k: line[k]["solves_per_s"] / line["c4_fp64"]["solves_per_s"]
            for k in ("c4", "c4_bf16_scms", "c4_refinement")}
        print("bench: 64-column p = 6 batch timed (float64 cycle)", file=sys.stderr, flush=True)
    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        line["calibration_copy_bytes"] = n * 8
    traffic_file = os.path.join(ROOT, "profiles", "traffic_%s_c2_fp64.json" % family)
    if os.path.exists(traffic_file):
        with open(traffic_file) as fh:
            tr = json.load(fh)
        # counters taken on the same kernel source and workload (checked by hash)
        if tr.get("source_hash") == source_hash(family) and tr.get("traffic_bytes"):
            roof["traffic"] = tr["traffic_bytes"]
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(cfg, f_host, its)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
