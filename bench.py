"""Benchmark: solves/s to relative residual 1e-8 on one MI355X, mixed
precision against float64, with the roofline position of the dominant kernel
and the FP64 CPU oracle timed on the host beside it.

Headline workload (the 64-column degree-6 configuration): 2D SIPG on the unit
square split into 4x4 bilinear patches (corners perturbed by up to 10% of the
patch width, seed 1902), 256 elements per patch direction, degree 6, penalty
5 p^2/h, 1,094,116 unknowns, 64 N(0,1) right-hand sides (seeds 4000..4063)
solved together; hybrid V(1,1) cycle (forward Gauss-Seidel + SCMS / SCMS +
backward Gauss-Seidel, damping 0.25, scaling 0.1) in float32 (operator rows,
smoother, transfers), float64 iterative refinement (float64 residual, update
and stopping test; coarse solve float64).  One step = one complete solve of
the 64 columns; the right-hand sides are resident in HBM before the timed
region starts; value = right-hand sides solved per second.

Beside it: the same batch with the float64 cycle (float64 PCG: the
mixed-vs-float64 speedup), flexible CG around the float32 cycle, bf16 SCMS
operands; the 3D workload (1.65 M unknowns) with float32 and float64 cycles;
the 4x4 degree-4 workload (115,652 unknowns) in float64 and float32; a
serving sample (p50/p99 latency).

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--quick]
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
                    "scms": "fdw_kernel", "iface_apply": "iface_kernel",
                    "stencil_apply": "sp2d_kernel", "outer_apply": "sp2d_kernel",
                    "stencil_rows": "sp2d_rhs_kernel"}


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


def cpu_baseline(cfg_name, scale, n_full, budget_s=15.0):
    """The oracle (plain FP64 CPU reference, as it stands) on a bounded sample
    of the headline workload: the same layout with every element count
    divided by `scale`, one right-hand side, float64 PCG solves to 1e-8
    repeated for about budget_s seconds (setup excluded, as on the GPU).  The
    rate is scaled to the full size by the ratio of unknowns (the solve's work
    is linear in the unknowns at a flat iteration count) and reported per
    right-hand side."""
    import oracle
    import workloads
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = 1
    cfg = workloads.config(cfg_name, scale)
    pb = oracle.setup(cfg["corners"], cfg["elems"], cfg["p"], sigma=cfg["sigma"],
                      conforming=cfg["conforming"], smoother=cfg["smoother"], tau=cfg["tau"],
                      delta=cfg["delta"])
    f = workloads.normal_rhs(pb.N, 4000)
    n = 0
    t0 = time.perf_counter()
    its = None
    while True:
        _, its, _, _ = pb.pcg(f)
        n += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    ratio = n_full / pb.N
    return dict(value=n / dt / ratio, unit="solves/s", cores=int(threads), kind="oracle",
                sample="%d float64 PCG solve(s) of the headline layout with element counts / %d "
                       "(%d unknowns, one right-hand side, %d iterations each, setup excluded) in "
                       "%.1f s; rate scaled to %d unknowns by the ratio of unknowns (%.1f)"
                       % (n, scale, pb.N, its, dt, n_full, ratio),
                measured_solves_per_s=n / dt, iterations=its, cpu_model=_cpu_model())


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


ROOF_FAMILIES = ("gauss_seidel", "stencil_apply", "stencil_rows", "outer_apply", "scms", "pieces",
                 "restrict", "prolong", "coarse", "vol_apply")


def family_times(st):
    fams = {}
    for key, v in st.items():
        fam = key.split("/")[0]
        fams[fam] = fams.get(fam, 0.0) + v["ms"]
    return fams


def roofline_entry(sv, family, level, nrhs, avg_s, precision):
    """Achieved rate of one launch of a kernel family against its roofline:
    algorithmic bytes (or flops) per launch from the library's model divided
    by the event-timed average launch."""
    mbytes, mflops = sv.kernel_model(family, level, nrhs)
    if family == "vol_apply":
        ach = mflops / avg_s / 1e12
        roof = dict(bound="alu", achieved=ach, peak=PEAK["fp64" if precision == "fp64" else "fp32"],
                    unit="TFLOP/s")
    elif family == "scms":
        ach = mflops / avg_s / 1e12
        roof = dict(bound="mfma", achieved=ach,
                    peak=MFMA_PEAK["bf16" if precision == "bf16" else precision], unit="TFLOP/s")
    else:
        ach = mbytes / avg_s / 1e9
        roof = dict(bound="hbm", achieved=ach, peak=PEAK["hbm"], unit="GB/s")
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["model_bytes_per_launch"] = mbytes
    roof["model_flops_per_launch"] = mflops
    return roof


def c4_solver(igamg, workloads, precision, outer, nrhs=64):
    cfg = workloads.config("c4")
    t0 = time.perf_counter()
    sv = igamg.Solver(cfg["corners"], cfg["elems"], cfg["p"], cfg["sigma"],
                      conforming=cfg["conforming"], smoother=cfg["smoother"], tau=cfg["tau"],
                      delta=cfg["delta"], precision=precision, outer=outer, max_rhs=nrhs)
    return cfg, sv, time.perf_counter() - t0


def c4_rhs(torch, workloads, n, nrhs=64, seed=4000):
    return torch.from_numpy(np.stack([workloads.normal_rhs(n, seed + j) for j in range(nrhs)])).cuda()


def timed_solves(torch, sv, F, U, steps, warmup):
    for _ in range(warmup):
        sv.solve(F, U, tol=1e-8, maxit=200)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for _ in range(steps):
        _, info = sv.solve(F, U, tol=1e-8, maxit=200)
        infos.append(info)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, infos


def column_errors(torch, U, Uref):
    """Relative error of every column of U against Uref (max, median)."""
    d = torch.linalg.norm(U - Uref, dim=1) / torch.linalg.norm(Uref, dim=1)
    d = d.cpu().numpy()
    return dict(max=float(d.max()), median=float(np.median(d)))


def finest_kernels(torch, sv, F, U, nrhs, precision):
    """Every modelled kernel family of the finest level in one more,
    event-timed solve: mean launch time and rate against its roofline."""
    top = sv.n_levels - 1
    sv.set_timing("")
    sv.solve(F, U, tol=1e-8, maxit=200)
    torch.cuda.synchronize()
    st = sv.kernel_stats(reset=True)
    sv.set_timing(None)
    out = {}
    for fam in ROOF_FAMILIES:
        k = "%s/%d" % (fam, 0 if fam == "coarse" else top)
        if not st.get(k, {}).get("launches"):
            continue
        t = st[k]["ms"] / 1e3 / st[k]["launches"]
        r = roofline_entry(sv, fam, top, nrhs, t, precision)
        out[fam] = dict(avg_us=t * 1e6, launches=st[k]["launches"], bound=r["bound"],
                        achieved=r["achieved"], unit=r["unit"], frac=r["frac"])
    out["ms_per_family_all_levels"] = {k: round(v, 3) for k, v in sorted(family_times(st).items())}
    return out


def c4_leg(igamg, torch, workloads, precision, outer, steps=2, warmup=1, Uref=None):
    """The 64 columns of the degree-6 workload with the given cycle
    arithmetic and outer iteration: rate, iterations, true residuals, kernel
    rates of the finest level, error per column against Uref."""
    cfg, sv, setup_s = c4_solver(igamg, workloads, precision, outer)
    F = c4_rhs(torch, workloads, sv.n_dofs)
    U = torch.zeros_like(F)
    dt, infos = timed_solves(torch, sv, F, U, steps, warmup)
    info = infos[-1]
    its = [i["iterations"] for i in info]
    out = dict(precision=precision, outer=outer, solves_per_s=F.shape[0] / dt,
               ms_per_batch=dt * 1e3, setup_s=setup_s, memory_gib=sv.memory() / (1 << 30),
               iterations_max=max(its), iterations_min=min(its),
               max_true_rel_residual=max(i["true_rel_residual"] for i in info),
               all_converged=all(i["converged"] and i["true_rel_residual"] <= 1e-8 for i in info))
    if Uref is not None:
        out["rel_error_vs_fp64_solution"] = column_errors(torch, U, Uref)
    out["kernels_finest"] = finest_kernels(torch, sv, F, U, F.shape[0], precision)
    sv.close()
    return out, U


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


def c3_leg(igamg, torch, workloads, precision="fp32", steps=2, operator_apply="auto", uref=None):
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
    u = torch.zeros_like(f)
    dt, infos = timed_solves(torch, sv, f, u, steps, 1)
    info = infos[-1]
    out = dict(workload="3D SIPG, 2x2x2 trilinear patches, 48/64 elements, p=3, manufactured",
               dofs=sv.n_dofs, levels=sv.n_levels, precision=precision, outer=outer,
               operator_apply=operator_apply,
               solves_per_s=1.0 / dt, ms_per_solve=dt * 1e3, setup_s=setup_s,
               memory_gib=sv.memory() / (1 << 30), iterations=info[0]["iterations"],
               true_rel_residual=info[0]["true_rel_residual"],
               converged=info[0]["converged"] and info[0]["true_rel_residual"] <= 1e-8,
               l2_error_manufactured=sv.l2_error(u))
    if uref is not None:
        out["rel_error_vs_fp64_solution"] = float(torch.linalg.norm(u - uref) /
                                                  torch.linalg.norm(uref))
    out["kernels_finest"] = finest_kernels(torch, sv, f, u, 1, precision)
    sv.close()
    return out, u


def _printed(name):
    """Iteration counts a table of the paper prints (tests/golden fixture):
    {L: row} with None where the paper prints no count."""
    rows = {}
    with open(os.path.join(ROOT, "tests", "golden", name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                v = [None if x == "-" else int(x) for x in line.split()]
                rows[v[0]] = v[1:]
    return rows


PAPER_TABLES = ("GS1", "SCMS1", "SCMS2", "HYB3a", "HYB3b")


def paper_tables(igamg, torch, workloads, maxit=150, tables=PAPER_TABLES):
    """The paper's L-shape and Fichera experiments on the GPU, each count
    beside the printed one: Table GS1 (L-shape, conforming, Gauss-Seidel
    V-cycle, multigrid used directly and as PCG preconditioner; L = 4..8,
    p = 2..8), Table SCMS1 (the same with the SCMS V-cycle, damping 1,
    scaling 0.12), Table SCMS2 (SIPG on the L-shape with the non-matching
    spaces S_{p,h}, S_{p+1,2h}, S_{p,2h}, SCMS V-cycle, scaling 0.12, the
    paper's damping 0.9 and 0.5; p = 2..7, degree p+1 = 9 being beyond the
    library's degree range) and Table HYB3 (a) (Fichera corner, hybrid
    V-cycle with PCG, scaling 0.12, L = 2..5, p = 2..4; damping 0.5, the
    largest for which this build's reading of the piece smoother keeps the
    cycle positive, and the paper's 1) and Table HYB3 (b) (the same with the
    SIPG space and the non-matching spaces; p = 2, 3: degree p+1 <= 4, the
    3D kernels' range).  A count of None means no convergence within maxit
    cycles."""
    out = {}

    def run(corners, elems, p, smoother, tau, outer, conforming=True):
        t0 = time.perf_counter()
        sv = igamg.Solver(corners, elems, p, 5.0, conforming=conforming, smoother=smoother,
                          tau=tau, delta=0.12, coarse_min=1, outer=outer)
        setup = time.perf_counter() - t0
        f = sv.load_manufactured()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u, info = sv.solve(f, tol=1e-8, maxit=maxit)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ok = info[0]["converged"] and info[0]["true_rel_residual"] <= 1e-8
        rec = dict(iterations=info[0]["iterations"] if ok else None, solve_s=dt, setup_s=setup,
                   dofs=sv.n_dofs)
        sv.close()
        return rec

    for table, smoother, tau, golden in (("GS1", "gs", 0.25, "gs1_lshape_conforming.txt"),
                                         ("SCMS1", "scms", 1.0, "scms1_lshape_conforming.txt")):
        if table not in tables:
            continue
        printed = _printed(golden)
        rows = []
        for L in range(4, 9):
            for p in range(2, 9):
                for blk, outer in (("a", "mg"), ("b", "pcg")):
                    col = (p - 2) + (0 if blk == "a" else 7)
                    r = run(workloads.lshape_corners(), workloads.lshape_elems(L), p, smoother,
                            tau, outer)
                    r.update(L=L, p=p, block=blk, printed=printed[L][col])
                    rows.append(r)
        out[table] = rows
        print("bench: table %s done" % table, file=sys.stderr, flush=True)
    if "SCMS2" in tables:
        printed = _printed("scms2_lshape_nonmatching.txt")
        rows = []
        for tau in (0.9, 0.5):
            for L in range(4, 9):
                for p in range(2, 8):
                    elems, deg = workloads.nonmatching_spaces(workloads.lshape_elems(L), p)
                    for blk, outer in (("a", "mg"), ("b", "pcg")):
                        col = (p - 2) + (0 if blk == "a" else 7)
                        r = run(workloads.lshape_corners(), elems, deg, "scms", tau, outer,
                                conforming=False)
                        r.update(L=L, p=p, block=blk, damping=tau, printed=printed[L][col])
                        rows.append(r)
        out["SCMS2"] = rows
        print("bench: table SCMS2 done", file=sys.stderr, flush=True)
    if "HYB3b" in tables:
        printed = _printed("hyb3_fichera.txt")
        rows = []
        for tau in (0.5, 1.0):
            for L in range(2, 6):
                for p in (2, 3):
                    elems, deg = workloads.nonmatching_spaces(workloads.fichera_elems(L), p)
                    r = run(workloads.fichera_corners(), elems, deg, "hybrid", tau, "pcg",
                            conforming=False)
                    r.update(L=L, p=p, block="b", damping=tau, printed=printed[L][5 + p - 2])
                    rows.append(r)
        out["HYB3b"] = rows
        print("bench: table HYB3 (b) done", file=sys.stderr, flush=True)
    if "HYB3a" not in tables:
        return out
    printed = _printed("hyb3_fichera.txt")
    rows = []
    for tau in (0.5, 1.0):
        for L in range(2, 6):
            for p in range(2, 5):
                r = run(workloads.fichera_corners(), workloads.fichera_elems(L), p, "hybrid",
                        tau, "pcg")
                r.update(L=L, p=p, block="a", damping=tau, printed=printed[L][p - 2])
                rows.append(r)
    out["HYB3a"] = rows
    print("bench: table HYB3 (a) done", file=sys.stderr, flush=True)
    return out


def c2_legs(igamg, torch, workloads, steps=10, warmup=2, coarse_min=8):
    """The 4x4 degree-4 workload (115,652 unknowns, one right-hand side):
    float64 PCG and the float32 cycle inside float64 flexible CG."""
    cfg = workloads.config("c2")
    out = {}
    u64 = None
    for precision, outer in (("fp64", "pcg"), ("fp32", "fcg")):
        sv = igamg.Solver(cfg["corners"], cfg["elems"], cfg["p"], cfg["sigma"],
                          conforming=cfg["conforming"], smoother=cfg["smoother"], tau=cfg["tau"],
                          delta=cfg["delta"], precision=precision, outer=outer,
                          coarse_min=coarse_min)
        f = torch.from_numpy(workloads.normal_rhs(sv.n_dofs, cfg["rhs"][1])).cuda()
        u = torch.zeros_like(f)
        dt, infos = timed_solves(torch, sv, f, u, steps, warmup)
        info = infos[-1]
        ent = dict(workload="2D SIPG, 4x4 bilinear patches, 64/96 elements, p=4, %d levels"
                            % sv.n_levels, dofs=sv.n_dofs, precision=precision, outer=outer,
                   solves_per_s=1.0 / dt, ms_per_solve=dt * 1e3,
                   iterations=info[0]["iterations"],
                   vcycles_per_s=(info[0]["iterations"] + 1) / dt,
                   true_rel_residual=info[0]["true_rel_residual"],
                   converged=all(i[0]["converged"] and i[0]["true_rel_residual"] <= 1e-8
                                 for i in infos))
        if u64 is not None:
            ent["rel_error_vs_fp64_solution"] = float(torch.linalg.norm(u - u64) /
                                                      torch.linalg.norm(u64))
        else:
            u64 = u.clone()
        ent["kernels_finest"] = finest_kernels(torch, sv, f, u, 1, precision)
        out[precision] = ent
        sv.close()
    out["fp32"]["speedup_vs_fp64"] = out["fp32"]["solves_per_s"] / out["fp64"]["solves_per_s"]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--quick", action="store_true",
                    help="headline and its float64 leg only (no 3D, degree-4, bf16, serving legs)")
    ap.add_argument("--serve-budget-gib", type=float, default=64.0,
                    help="device memory the serving runtime admits requests into")
    ap.add_argument("--serve-requests", type=int, default=96,
                    help="requests of the serving sample (0 = skip)")
    ap.add_argument("--c1-only", action="store_true",
                    help="diagnostic: run only the conforming 2x2 workload (rates, a batch of "
                         "1000 right-hand sides, L2 error ladder) and print its results")
    ap.add_argument("--c3-only", action="store_true",
                    help="diagnostic: run only the full-size 3D legs and print their results")
    ap.add_argument("--paper-tables", nargs="?", const=",".join(PAPER_TABLES), default=None,
                    metavar="T1,T2",
                    help="run only the paper's L-shape and Fichera experiments (Tables GS1, "
                         "SCMS1, SCMS2, HYB3a, HYB3b; default all) and print the counts beside the "
                         "printed ones")
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

    def note(msg):
        print("bench: " + msg, file=sys.stderr, flush=True)

    if args.c1_only:
        print(json.dumps({"c1": c1_leg(igamg, torch, workloads)}))
        return

    if args.paper_tables:
        tabs = tuple(t for t in args.paper_tables.split(",") if t)
        bad = [t for t in tabs if t not in PAPER_TABLES]
        if bad:
            print("unknown table(s) %s; choose from %s" % (bad, PAPER_TABLES), file=sys.stderr)
            sys.exit(2)
        print(json.dumps(paper_tables(igamg, torch, workloads, tables=tabs)))
        return

    if args.c3_only:
        o64, u64 = c3_leg(igamg, torch, workloads, precision="fp64")
        note("3D workload timed (float64 cycle)")
        o32, _ = c3_leg(igamg, torch, workloads, precision="fp32", uref=u64)
        note("3D workload timed (float32 cycle)")
        obf, _ = c3_leg(igamg, torch, workloads, precision="bf16", uref=u64)
        out = {"c3_fp64": o64, "c3_fp32": o32, "c3_bf16_scms": obf,
               "mixed_speedup": {"fp32": o32["solves_per_s"] / o64["solves_per_s"],
                                 "bf16_scms": obf["solves_per_s"] / o64["solves_per_s"]}}
        print(json.dumps(out))
        return

    # ---- headline: 64 columns, float32 cycle in float64 iterative refinement
    precision, outer, nrhs = "fp32", "ir", 64
    cfg, sv, setup_s = c4_solver(igamg, workloads, precision, outer, nrhs)
    N = sv.n_dofs
    F = c4_rhs(torch, workloads, N, nrhs)
    U = torch.zeros_like(F)
    for _ in range(args.warmup):
        sv.solve(F, U, tol=1e-8, maxit=200)
    torch.cuda.synchronize()
    top = sv.n_levels - 1
    family = args.family
    if family is None:
        # the family with the most event time over all levels in one
        # instrumented (untimed) solve
        sv.set_timing("")
        sv.solve(F, U, tol=1e-8, maxit=200)
        fams = family_times(sv.kernel_stats(reset=True))
        family = max([k for k in ROOF_FAMILIES if k in fams], key=lambda k: fams[k])
        # a float32 batch applies the operator with three kernels: the entry
        # is the row kernel's (its own event family)
        if family == "stencil_apply" and "stencil_rows" in fams:
            family = "stencil_rows"
    # timed region: only the dominant family's finest-level launches carry
    # events (on the library's stream, where the kernels run)
    key = "%s/%d" % (family, 0 if family == "coarse" else top)
    sv.set_timing(key)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for _ in range(args.steps):
        _, info = sv.solve(F, U, tol=1e-8, maxit=200)
        infos.append(info)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = sv.kernel_stats(reset=True)
    sv.set_timing(None)
    note("headline timed (%.1f ms per batch of %d)" % (dt / args.steps * 1e3, nrhs))
    launches = st[key]["launches"]
    avg_s = st[key]["ms"] / 1e3 / max(launches, 1)
    roof = roofline_entry(sv, family, top, nrhs, avg_s, precision)
    roof.update(traffic=None, kernel=key, avg_launch_us=avg_s * 1e6, launches=launches,
                units_per_launch=("one colour class of a Gauss-Seidel sweep on the finest level "
                                  "(the sweep's stencil rows and vectors split evenly over its "
                                  "class launches), %d right-hand sides" % nrhs)
                if family == "gauss_seidel" else
                "one launch on the finest level, %d right-hand sides" % nrhs)
    kernels = finest_kernels(torch, sv, F, U, nrhs, precision)
    last = infos[-1]
    value = nrhs * args.steps / dt
    its = [i["iterations"] for i in last]
    ok = all(i["converged"] and i["true_rel_residual"] <= 1e-8 for info in infos for i in info)
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
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "2D SIPG, 4x4 bilinear patches (10%% seeded perturbation), 256 "
                               "elements per patch direction, p=6, sigma=5, %d N(0,1) right-hand "
                               "sides solved together; hybrid V(1,1) over %d levels in float32 "
                               "(float64 coarse solve) inside float64 iterative refinement to "
                               "rel. residual 1e-8" % (nrhs, sv.n_levels),
                   "dofs": N, "nrhs": nrhs, "levels": sv.n_levels,
                   "cycle_dtype": "f32", "outer_dtype": "f64", "outer": "iterative refinement",
                   "iterations_max": max(its), "iterations_min": min(its),
                   "batch_vcycles_per_s": args.steps * float(np.mean(its)) / dt,
                   "max_true_rel_residual": max(i["true_rel_residual"] for i in last),
                   "all_converged": ok, "setup_s": setup_s,
                   "memory_gib": sv.memory() / (1 << 30)},
        "roofline": roof,
        "kernels_finest": kernels,
    }
    sv.close()
    Umixed = U
    # ---- float64 cycle on the same batch (float64 PCG): the speedup's base
    o64, U64 = c4_leg(igamg, torch, workloads, "fp64", "pcg", steps=2, warmup=1)
    note("float64 batch timed")
    line["fp64"] = o64
    line["config"]["rel_error_vs_fp64_solution"] = column_errors(torch, Umixed, U64)
    line["mixed_speedup_vs_fp64"] = value / o64["solves_per_s"]
    del Umixed
    if not args.quick:
        for name, prec, out_ in (("fcg_fp32", "fp32", "fcg"), ("ir_bf16_scms", "bf16", "ir")):
            o, _ = c4_leg(igamg, torch, workloads, prec, out_, steps=2, warmup=1, Uref=U64)
            o["speedup_vs_fp64"] = o["solves_per_s"] / o64["solves_per_s"]
            line[name] = o
            note("%s batch timed" % name)
    del U64
    torch.cuda.empty_cache()
    if not args.quick:
        c3_64, u3 = c3_leg(igamg, torch, workloads, precision="fp64")
        note("3D workload timed (float64 cycle)")
        c3_32, _ = c3_leg(igamg, torch, workloads, precision="fp32", uref=u3)
        note("3D workload timed (float32 cycle)")
        c3_32["speedup_vs_fp64"] = c3_32["solves_per_s"] / c3_64["solves_per_s"]
        line["c3"] = {"fp64": c3_64, "fp32": c3_32}
        del u3
        torch.cuda.empty_cache()
        line["c2"] = c2_legs(igamg, torch, workloads)
        note("degree-4 workload timed")
        if args.serve_requests > 0:
            from paper_1902_01818_amd import serve
            line["serving"] = serve.serve_benchmark(
                n_requests=args.serve_requests, slots=4, budget_gib=args.serve_budget_gib,
                load=0.7, calibrate=min(max(32, args.serve_requests // 16), args.serve_requests))
            note("serving sample done")
    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        line["calibration_copy_bytes"] = n * 8
    traffic_file = os.path.join(ROOT, "profiles", "traffic_%s_c4_ir.json" % family)
    if os.path.exists(traffic_file):
        with open(traffic_file) as fh:
            tr = json.load(fh)
        # counters taken on the same kernel source and workload (checked by hash)
        if (family in KERNEL_OF_FAMILY and tr.get("source_hash") == source_hash(family)
                and tr.get("traffic_bytes")):
            roof["traffic"] = tr["traffic_bytes"]
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline("c4", 8, N)
        note("cpu baseline done")
    print(json.dumps(line))


if __name__ == "__main__":
    main()
