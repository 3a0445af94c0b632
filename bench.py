"""Benchmark of the multipole Poisson solve on one MI355X.

One step = one full solve (density streaming, moment contraction, split-K
sum, radial scans and coefficients, expansion contraction and potential
streaming) of a synthetic density already resident in HBM.  Prints one JSON
line with throughput in cell*(l,m)-modes/s (fine cells x (lmax+1)^2 per
second), the roofline position of the dominant kernel measured with HIP
events inside the timed region, and the FP64 CPU oracle timed on the host.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell*(l,m)-modes/s, multipole Phi solve: mixed vs FP64 on GPU at <=1e-6 rel err"
UNIT = "cell*(l,m)-modes/s"
PEAK = {"f64": (78.6e12, "TFLOP/s"), "bf16": (2.5e15, "TFLOP/s"), "f16": (2.5e15, "TFLOP/s")}
DTYPE = {"fp64": "f64", "bf16x3": "bf16", "fp16x2": "f16", "fp64sep": "f64", "bf16x3sep": "bf16"}

WORKLOADS = {
    # name: (workload generator key, precision)
    "production_fp64": ("production", "fp64"),
    "production_bf16x3": ("production", "bf16x3"),
    "production_l32_fp64": ("production_l32", "fp64"),
    "production_l32_bf16x3": ("production_l32", "bf16x3"),
    "production_l32_fp16x2": ("production_l32", "fp16x2"),
    # separable FP64 contractions (phi transform + per-m theta transforms)
    "production_sep": ("production", "fp64sep"),
    "production_l32_sep": ("production_l32", "fp64sep"),
    # separable with BF16 x3 phi transforms (m >= 1), FP64 theta transforms
    "production_l32_bf16x3sep": ("production_l32", "bf16x3sep"),
    "spheroid_fp64": ("spheroid", "fp64"),
    # 64 uneven fields, one launch per phase, replayed from a HIP graph
    "batch64_bf16x3": ("batch64", "bf16x3"),
    "batch64_fp64": ("batch64", "fp64"),
    "batch64_sep": ("batch64", "fp64sep"),
    # 2048 x 256 x 512, lmax 64: --steps consecutive solves (1000 for the full
    # run) on a rotating density, density update + solve per step, one HIP graph
    "large_fp16x2": ("large", "fp16x2"),
    "large_bf16x3": ("large", "bf16x3"),
    "large_sep": ("large", "fp64sep"),
    "large_bf16x3sep": ("large", "bf16x3sep"),
    # GenASiS mesh of the spheroid tests (N_theta 256, r_core 0.25, R_radial 3.68:
    # 942 x 256 x 512, 201 coarsening classes), lmax 12 (the paper's default)
    "genasis_sep": ("genasis", "fp64sep"),
    "genasis_bf16x3": ("genasis", "bf16x3"),
    "genasis_bf16x3sep": ("genasis", "bf16x3sep"),
    "batch64_bf16x3sep": ("batch64", "bf16x3sep"),
}
DEFAULT = "production_l32_bf16x3"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default=DEFAULT, choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true", help="skip the oracle comparison")
    ap.add_argument("--no-fp64", action="store_true", help="skip timing the FP64 path beside a split precision")
    ap.add_argument("--no-tune", action="store_true", help="default launch tuning instead of the autotuner's")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 5 device-to-device copies of MIB MiB (reference for HBM byte counters)")
    return ap.parse_args()


KERNEL_NAMES = {("fp64", "moment"): "k_moment_f64", ("fp64", "expand"): "k_expand_f64",
                ("fp64sep", "moment"): "k_sep_phi_anal", ("fp64sep", "expand"): "k_sep_phi_syn",
                ("bf16x3sep", "moment"): "k_sep_phi_anal_bf16", ("bf16x3sep", "expand"): "k_sep_phi_syn_bf16"}


def kernel_name(precision, phase):
    if (precision, phase) in KERNEL_NAMES:
        return KERNEL_NAMES[(precision, phase)]
    return "k_gemm_split<%s, %s>" % (precision, phase)


def sources_sha256_16(sources):
    """First 16 hex digits of the sha256 of the named files, concatenated in
    order (None if one is missing): the kernel sources a counter entry holds
    for."""
    import hashlib
    h = hashlib.sha256()
    for s in sources:
        path = os.path.join(ROOT, s)
        if not os.path.exists(path):
            return None
        h.update(open(path, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(workload, phase):
    """HBM bytes per launch from the committed counter runs, or None when there
    is none for this kernel or its source changed since they were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_counters.json")
    if not os.path.exists(path):
        return None
    data = json.load(open(path))
    cal = data["copy_calibration"]
    for e in data["entries"]:
        if e["workload"] != workload or e["phase"] != phase:
            continue
        if sources_sha256_16(e["sources"]) != e["sha256_16"]:
            return None
        return 1024.0 * (cal["fetch_factor"] * e["fetch_kib"] + cal["write_factor"] * e["write_kib"])
    return None


def copy_calibration(mib):
    """Plain copies of known size, so that the FETCH_SIZE / WRITE_SIZE counters
    of one dispatch can be converted to bytes: each copy reads and writes
    exactly mib MiB."""
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print("copy calibration: 5 copies of %d MiB" % mib, flush=True)


def roofline_hbm(plan, phases, workload):
    """Roofline of the BF16 x3 separable path, whose phi transforms are bound
    by HBM: algorithmic bytes of the dominant transform / its phase duration
    (the synthesis phase includes the block means of the potential) against
    the HBM peak.  Analysis: the density read once (8 B per cell) and F
    written ((2L+1) x ntheta x 8 B per shell); synthesis: G read and the
    potential written once."""
    dom = max(("moment", "expand"), key=lambda k: phases[k][0])
    dom_ms = phases[dom][0] / max(phases[dom][1], 1)
    cells = float(plan.nr) * plan.shape[1] * plan.shape[2]
    modes = (2 * plan.lmax + 1) * float(plan.nr) * plan.shape[1]
    nbytes = 8.0 * cells + 8.0 * modes
    achieved = nbytes / (dom_ms * 1e-3)
    # meshes of whole K steps (nphi % 32) and whole tile pairs (also ntheta %
    # 64 for the synthesis) run the whole-tile forms of the transforms
    full = plan.shape[2] % 32 == 0 and (dom == "moment" or plan.shape[1] % 64 == 0)
    kernel = kernel_name("bf16x3sep", dom) + ("_full" if full else "")
    return {"bound": "hbm", "kernel": kernel, "achieved": achieved / 1e9, "peak": 8000.0,
            "unit": "GB/s", "frac": achieved / 8e12, "traffic": measured_traffic(workload, dom), "launch_ms": dom_ms,
            "algorithmic_bytes_per_launch": nbytes,
            "phase_ms": {k: v[0] / max(v[1], 1) for k, v in phases.items() if v[1]}}


def solve_bound(plan, precision, ms):
    """Whole-solve roofline: the sum over the solve's phases of max(executed
    flops / the peak of their arithmetic, algorithmic bytes / the HBM peak),
    set against the measured time per solve.  Bytes: the density read and the
    potential written once (8 B per cell each), each narrow or FP64 operand
    written and read once, the kernel table read once per contraction, the
    moments, edge sums and coefficients once each; flops: 2 per multiply-add,
    times the narrow products per multiply-add."""
    hbm = 8e12
    f64 = PEAK["f64"][0]
    nr, nt, nph = plan.nr, plan.shape[1], plan.shape[2]
    cells = float(nr) * nt * nph
    nam = (plan.lmax + 1) ** 2
    mflops, eflops, min_bytes = plan.work()
    # a folded plan contracts block pairs: half the multiply-adds and half the
    # kernel table of the algorithmic count
    fold = 0.5 if getattr(plan, "folded", False) else 1.0
    scan_bytes = 8.0 * nam * (nr + 3 * (nr + 1))
    t = {}
    if precision in ("fp64sep", "bf16x3sep"):
        inter = 8.0 * (2 * plan.lmax + 1) * nr * nt   # F or G, [shell][trig mode][theta]
        peak = PEAK[DTYPE[precision]][0]
        prod = 6 if precision == "bf16x3sep" else 1
        theta_flops = 2.0 * nr * nt * nam
        t["phi_analysis"] = max(mflops * prod / peak, (8.0 * cells + inter) / hbm)
        t["theta_analysis"] = max(theta_flops / f64, (inter + 8.0 * nr * nam) / hbm)
        t["scan"] = scan_bytes / hbm
        t["theta_synthesis"] = max(theta_flops / f64, (8.0 * nr * nam + inter) / hbm)
        t["phi_synthesis"] = max(eflops * prod / peak, (inter + 8.0 * cells) / hbm)
    else:
        peak = PEAK[DTYPE[precision]][0]
        prod = {"fp64": 1, "bf16x3": 6, "fp16x2": 3}[precision]
        opb = {"fp64": 8.0, "bf16x3": 6.0, "fp16x2": 4.0}[precision]   # bytes per operand element
        blocks = mflops / (2.0 * nam)                  # (shell, merged block) pairs
        table = (min_bytes - 16.0 * cells) * opb / 8.0 * fold
        t["pack"] = (8.0 * cells + opb * blocks) / hbm
        t["moment"] = max(mflops * fold * prod / peak, (opb * blocks + table) / hbm)
        t["scan"] = scan_bytes / hbm
        t["expand"] = max(eflops * fold * prod / peak, (table + 8.0 * cells) / hbm)
    bound = sum(t.values()) * 1e3
    return {"bound_ms": bound, "measured_ms": ms, "frac": bound / ms,
            "phase_bound_ms": {k: v * 1e3 for k, v in t.items()}}


def roofline(plan, phases, precision, workload):
    """Roofline position of the dominant contraction from the plan's per-phase
    HIP event timings: algorithmic flops of one launch / its mean duration
    against the MFMA peak of the arithmetic type."""
    if precision == "bf16x3sep":
        return roofline_hbm(plan, phases, workload)
    mflops, eflops, _ = plan.work()
    dom = max(("moment", "expand"), key=lambda k: phases[k][0])
    dom_ms = phases[dom][0] / max(phases[dom][1], 1)
    flops = mflops if dom == "moment" else eflops
    peak, punit = PEAK[DTYPE[precision]]
    achieved = flops / (dom_ms * 1e-3)
    # executed MFMA work: the split precisions run `products` narrow products per
    # algorithmic multiply-add, over padded tiles
    products = {"fp64": 1, "bf16x3": 6, "fp16x2": 3, "fp64sep": 1, "bf16x3sep": 6}[precision]
    # a folded plan executes half the algorithmic multiply-adds (block pairs)
    fold = 0.5 if getattr(plan, "folded", False) else 1.0
    kernel = kernel_name(precision, dom)
    # the FP64 separable synthesis on 64 x 64 tiles with 2L + 1 <= 100 runs its
    # whole-K form
    if precision == "fp64sep" and dom == "expand" and plan.shape[1] % 64 == 0 and plan.shape[2] % 64 == 0 \
            and (2 * plan.lmax + 4) // 4 <= 25:
        kernel += "_w"
    return {"bound": "mfma", "kernel": kernel,
            "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": punit, "frac": achieved / peak,
            "traffic": measured_traffic(workload, dom), "launch_ms": dom_ms,
            "algorithmic_flops_per_launch": flops, "narrow_products_per_madd": products,
            "mirror_fold": fold < 1.0, "executed_flops_per_launch": flops * fold * products,
            "executed_frac_lower_bound": achieved * fold * products / peak,
            "phase_ms": {k: v[0] / max(v[1], 1) for k, v in phases.items() if v[1]}}


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        sys.stderr.write("bench.py: this build runs on one GPU only; --gpus %d is not supported\n" % args.gpus)
        sys.exit(2)
    import torch
    from paper_2602_02507_amd import mpole
    from paper_2602_02507_amd import workloads as wl

    if not torch.cuda.is_available():
        sys.stderr.write("bench.py: no GPU visible\n")
        sys.exit(1)
    key, precision = WORKLOADS[args.workload]
    if key == "batch64":
        return bench_batch(args, precision)
    if key == "large":
        return bench_large(args, precision)
    if key == "genasis":
        # the mesh comes from the library's builder; the oracle is not run at
        # this size (its per-class kernel tables would need tens of GB of host
        # memory): the error is taken against the dense FP64 GPU path, which
        # the tests pin to the oracle on GenASiS meshes
        g = mpole.genasis_mesh(256, 0.25, 3.68, dims=3)
        mesh = wl.Mesh(g["r_edges"], g["theta_edges"], g["phi_edges"], 12, g["shell_class"], g["class_block"],
                       name="genasis")
        rho_h = wl.production_density(mesh, seed=2)
        args.no_check = args.no_cpu_baseline = True
    else:
        mesh, rho_h = wl.workload(key)
    dev = torch.device("cuda:0")
    print("bench: workload %s %dx%dx%d lmax %d precision %s" % (args.workload, mesh.nr, mesh.ntheta, mesh.nphi,
                                                                mesh.lmax, precision), file=sys.stderr, flush=True)
    rho = torch.from_numpy(rho_h).to(dev)
    stream = torch.cuda.current_stream(dev)

    # launch tuning from the autotuner (cached per device and mesh shape), outside the timed region
    tunings, tune_s = {}, 0.0
    if not args.no_tune:
        from paper_2602_02507_amd import tune
        t0 = time.perf_counter()
        for prec in ([precision] if precision == "fp64" or args.no_fp64 else [precision, "fp64"]):
            tunings[prec] = tune.tune_plan(mesh, prec, dev, log=lambda m: print("bench: " + m, file=sys.stderr,
                                                                                   flush=True))
        tune_s = time.perf_counter() - t0

    def time_path(prec):
        """Mean solve time of another precision path on the same workload (and its potential)."""
        p2 = mpole.Plan.from_mesh(mesh, precision=prec, device=dev, tuning=tunings.get(prec))
        o2 = p2.empty_outputs()
        for _ in range(args.warmup):
            p2.solve_into(rho, **o2)
        t = time_solves(lambda: p2.solve_into(rho, **o2), args.steps, stream)
        bound = solve_bound(p2, prec, t["graph_ms"])
        del p2
        return {"ms_per_step": t["graph_ms"], "eager_ms_per_step": t["eager_ms"], "phi": o2["phi"],
                "solve_roofline_frac": bound["frac"]}

    fp64 = None
    if precision != "fp64" and not args.no_fp64:
        # the plain FP64 GPU solve of the same workload, for the speedup figure
        fp64 = time_path("fp64")
        print("bench: fp64 path %.4f ms/solve" % fp64["ms_per_step"], file=sys.stderr, flush=True)
    # the separable forms of the same solve, reported beside the dense one
    others = {}
    if precision == "bf16x3" and fp64 is not None:
        for prec in ("bf16x3sep", "fp64sep"):
            r = time_path(prec)
            err = float((r["phi"] - fp64["phi"]).abs().div(fp64["phi"].abs()).max())
            others[prec] = {"ms_per_step": r["ms_per_step"], "speedup_vs_fp64": fp64["ms_per_step"] / r["ms_per_step"],
                            "max_rel_err_vs_fp64_gpu": err, "solve_roofline_frac": r["solve_roofline_frac"]}
            print("bench: %s path %.4f ms/solve, max rel err vs FP64 %.2e" % (prec, r["ms_per_step"], err),
                  file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = mpole.Plan.from_mesh(mesh, precision=precision, device=dev, tuning=tunings.get(precision))
    torch.cuda.synchronize()
    plan_ms = 1e3 * (time.perf_counter() - t0)   # plan creation + table build (not part of a solve)
    out = plan.empty_outputs()
    for _ in range(args.warmup):
        plan.solve_into(rho, **out)
    torch.cuda.synchronize()

    # the measured value: K solves captured in one HIP graph and replayed
    # (the eager launch rate and per-step spread come from the same call)
    t = time_solves(lambda: plan.solve_into(rho, **out), args.steps, stream)
    ms, step_ms, wall = t["graph_ms"], t["step_ms"], t["wall_s"]
    # per-kernel durations from the library's event pairs, in a separate
    # eager loop (the events add launch gaps of their own)
    plan.set_timing(True)
    plan.phase_ms()                     # clear
    for _ in range(min(args.steps, 20)):
        plan.solve_into(rho, **out)
    torch.cuda.synchronize()
    phases = plan.phase_ms()
    plan.set_timing(False)
    print("bench: %.4f ms/solve in a graph (eager %.4f, wall %.4f ms); phases %s" % (
        ms, t["eager_ms"], 1e3 * wall / args.steps,
        {k: round(v[0] / max(v[1], 1), 5) for k, v in phases.items() if v[1]}), file=sys.stderr, flush=True)

    cell_modes = float(mesh.ncells) * mesh.nmodes
    value = cell_modes / (ms * 1e-3)
    roof = roofline(plan, phases, precision, args.workload)
    roof["solve"] = solve_bound(plan, precision, ms)
    dtype = DTYPE[precision]

    # the gradient of the potential for the gravitational sources (after the
    # solve, not part of a step): HBM-bound, 8 B read + 24 B written per cell
    grads = [torch.empty_like(out["phi"]) for _ in range(3)]
    plan.gradient(out["phi"], *grads)
    g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    g0.record(stream)
    for _ in range(10):
        plan.gradient(out["phi"], *grads)
    g1.record(stream)
    torch.cuda.synchronize()
    grad_ms = g0.elapsed_time(g1) / 10
    del grads
    # the gravitational sources -rho grad Phi and -rho v . grad Phi in one
    # pass (synthetic velocity field): 40 B read + 32 B written per cell
    gen = torch.Generator(device=dev)
    gen.manual_seed(11)
    vel = [torch.randn(out["phi"].shape, dtype=torch.float64, device=dev, generator=gen) for _ in range(3)]
    srcs = tuple(torch.empty_like(out["phi"]) for _ in range(4))
    plan.gravity_sources(out["phi"], rho, tuple(vel), out=srcs)
    g0.record(stream)
    for _ in range(10):
        plan.gravity_sources(out["phi"], rho, tuple(vel), out=srcs)
    g1.record(stream)
    torch.cuda.synchronize()
    src_ms = g0.elapsed_time(g1) / 10
    del vel, srcs
    # the block volume average (coarsening operation) of the density into
    # another buffer: HBM-bound, 8 B read + 8 B written per cell
    work = torch.empty_like(rho)
    plan.coarsen(rho, out=work)
    g0.record(stream)
    for _ in range(10):
        plan.coarsen(rho, out=work)
    g1.record(stream)
    torch.cuda.synchronize()
    coarsen_ms = g0.elapsed_time(g1) / 10
    del work

    result = {"metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": args.steps,
              "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
              "vs_baseline": None, "dtype": dtype, "data": "synthetic",
              "config": {"workload": args.workload, "nr": mesh.nr, "ntheta": mesh.ntheta, "nphi": mesh.nphi,
                         "lmax": mesh.lmax, "precision": precision,
                         "coarsened": mesh.class_block is not None, "hip_graph": True},
              "roofline": roof,
              "eager_ms_per_step": t["eager_ms"],
              "step_ms_p50": float(np.percentile(step_ms, 50)), "step_ms_p99": float(np.percentile(step_ms, 99)),
              "plan_ms": plan_ms,
              "gradient": {"ms": grad_ms, "algorithmic_gbs": 32.0 * mesh.ncells / (grad_ms * 1e-3) / 1e9,
                           "hbm_frac": 32.0 * mesh.ncells / (grad_ms * 1e-3) / 8e12},
              "gravity_sources": {"ms": src_ms, "algorithmic_gbs": 72.0 * mesh.ncells / (src_ms * 1e-3) / 1e9,
                                  "hbm_frac": 72.0 * mesh.ncells / (src_ms * 1e-3) / 8e12},
              "coarsen": {"ms": coarsen_ms, "classes": 0 if mesh.class_block is None else int(mesh.class_block.shape[0]),
                          "algorithmic_gbs": 16.0 * mesh.ncells / (coarsen_ms * 1e-3) / 1e9,
                          "hbm_frac": 16.0 * mesh.ncells / (coarsen_ms * 1e-3) / 8e12},
              "tuning": plan.tuning(), "autotuned": not args.no_tune, "tune_s": tune_s}
    if fp64 is not None:
        result["fp64_ms_per_step"] = fp64["ms_per_step"]
        result["speedup_vs_fp64"] = fp64["ms_per_step"] / ms
        result["max_rel_err_vs_fp64_gpu"] = float((out["phi"] - fp64["phi"]).abs().div(fp64["phi"].abs()).max())
    if others:
        result["separable_paths"] = others

    if not (args.no_cpu_baseline and args.no_check):
        import oracle
        oracle.set_threads(host_threads())
        t0 = time.perf_counter()
        ref = oracle.solve(rho=rho_h, **mesh.oracle_kwargs())
        tot = time.perf_counter() - t0
        t_tables, t_solve = ref["seconds"]
        if not args.no_cpu_baseline:
            # repeated full solves of the same workload until about 10 s of
            # solve time have accumulated (the tables are built once per call
            # and excluded)
            reps, t_sum = 1, t_solve
            while t_sum < 10.0 and reps < 64:
                t_sum += oracle.solve(rho=rho_h, **mesh.oracle_kwargs())["seconds"][1]
                reps += 1
            result["cpu_baseline"] = {"value": reps * cell_modes / t_sum, "unit": UNIT, "cores": oracle.threads(),
                                      "kind": "oracle", "cpu_model": cpu_model(),
                                      "sample": "%d full solves of the same workload, %.2f s of solve time (tables "
                                                "excluded: %.2f s per call; first call %.2f s in all)"
                                                % (reps, t_sum, t_tables, tot),
                                      "single_thread": single_thread_rate(mesh, rho_h)}
        if not args.no_check:
            torch.cuda.synchronize()
            phi = out["phi"].cpu().numpy()
            result["max_rel_err_vs_oracle"] = float(np.max(np.abs(phi - ref["phi"]) / np.abs(ref["phi"])))
    print(json.dumps(result), flush=True)


def time_solves(solve, steps, stream):
    """Mean time of `steps` solves: eager launches between per-step events
    (mean, per-step spread), then the same solves captured in one HIP graph
    and replayed (warm replay first); the graph figure is the measured one."""
    import torch
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev[0].record(stream)
    for k in range(steps):
        solve()
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    eager_ms = ev[0].elapsed_time(ev[-1]) / steps
    step_ms = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)])
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(steps):
            solve()
    g.replay()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    g.replay()
    b.record(stream)
    torch.cuda.synchronize()
    graph_ms = a.elapsed_time(b) / steps
    del g
    return {"eager_ms": eager_ms, "graph_ms": graph_ms, "step_ms": step_ms, "wall_s": wall}


def cpu_model():
    """Model name of the host CPU (first entry of /proc/cpuinfo)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def host_threads():
    """Threads for the multi-threaded oracle leg: the CPUs this process may
    run on (the machine's CPU share, not the machine's core count)."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def single_thread_rate(mesh, rho_h, shells=64):
    """The oracle on one thread, on a bounded sample of the workload: one solve
    of its outermost `shells` shells (same angular mesh, lmax and coarsening
    class as there; the outer shells carry the most blocks per shell, so the
    rate is, if anything, below the full mesh's).  Thread count restored
    afterwards."""
    import oracle
    nr = mesh.nr
    s0 = max(0, nr - shells)
    sc = None if mesh.shell_class is None else np.ascontiguousarray(mesh.shell_class[s0:])
    from paper_2602_02507_amd import workloads as wl
    sub = wl.Mesh(mesh.r_edges[s0:], mesh.theta_edges, mesh.phi_edges, mesh.lmax, sc, mesh.class_block, mesh.G)
    prev = oracle.threads()
    oracle.set_threads(1)
    try:
        ref = oracle.solve(rho=np.ascontiguousarray(rho_h[s0:]), **sub.oracle_kwargs())
    finally:
        oracle.set_threads(prev)
    t = ref["seconds"][1]
    return {"value": float(sub.ncells) * sub.nmodes / t, "unit": UNIT, "cores": 1,
            "sample": "one solve of the outermost %d of %d shells on one thread, %.2f s (tables excluded)"
                      % (nr - s0, nr, t)}


def _tuning_summary(tunings):
    """Counts of the tile heights chosen over the fields and the moment workgroup total."""
    if not tunings:
        return None
    out = {"moment_wgs_total": int(sum(t["moment_wgs"] for t in tunings))}
    for k in ("moment_tile_m", "expand_tile_m"):
        vals, counts = np.unique([t[k] for t in tunings], return_counts=True)
        out[k] = {str(int(v)): int(c) for v, c in zip(vals, counts)}
    return out


def bench_large(args, precision):
    """Repeated solve on a large mesh: args.steps steps, each a density update
    (the l <= 8 perturbation rotated by the next seeded rotation, written on the
    device) and one solve, all captured in one HIP graph, with a copy of the
    potential kept every 100th step.  After the timed replay each kept
    potential is compared with the FP64 GPU solve of the same step's density."""
    import torch
    from paper_2602_02507_amd import devicegen, mpole
    from paper_2602_02507_amd import workloads as wl
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    mesh = wl.large_mesh()
    steps = args.steps
    every = min(100, steps)
    log = lambda m: print("bench: " + m, file=sys.stderr, flush=True)
    log("large workload %dx%dx%d lmax %d %s, %d steps" % (mesh.nr, mesh.ntheta, mesh.nphi, mesh.lmax, precision,
                                                          steps))
    coef = wl.real_ylm_coeffs(wl.LARGE_LPERT, wl.LARGE_SEED)
    gen = devicegen.RotatedDensity(mesh, coef, wl.rotation_sequence(steps), wl.LARGE_EPS, device=dev)
    rho = torch.empty(mesh.shape, dtype=torch.float64, device=dev)
    phi = torch.empty_like(rho)
    tuning, tune_s = None, 0.0
    if not args.no_tune:
        from paper_2602_02507_amd import tune
        t0 = time.perf_counter()
        tuning = tune.tune_plan(mesh, precision, dev, log=log)
        tune_s = time.perf_counter() - t0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = mpole.Plan.from_mesh(mesh, precision=precision, device=dev, tuning=tuning)
    torch.cuda.synchronize()
    plan_ms = 1e3 * (time.perf_counter() - t0)
    log("plan built in %.0f ms (workspace %.2f GB)" % (plan_ms, plan.workspace_bytes / 1e9))
    snaps = [torch.empty_like(rho) for _ in range(steps // every)]

    # density generator alone, and the per-phase split of an eager solve
    gen.write(rho, 0)
    for _ in range(max(args.warmup, 1)):
        plan.solve_into(rho, phi=phi)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(stream)
    for t in range(10):
        gen.write(rho, t % (steps + 1))
    b.record(stream)
    torch.cuda.synchronize()
    density_ms = a.elapsed_time(b) / 10
    gen.write(rho, 0)
    plan.set_timing(True)
    plan.phase_ms()
    for _ in range(3):
        plan.solve_into(rho, phi=phi)
    torch.cuda.synchronize()
    phases = plan.phase_ms()
    plan.set_timing(False)

    # one graph of `steps` consecutive steps
    t0 = time.perf_counter()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream(dev)
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            for t in range(1, steps + 1):
                gen.write(rho, t)
                plan.solve_into(rho, phi=phi)
                if t % every == 0:
                    snaps[t // every - 1].copy_(phi)
    stream.wait_stream(side)
    torch.cuda.synchronize()
    log("captured %d steps in %.1f s" % (steps, time.perf_counter() - t0))
    a.record(stream)
    g.replay()
    b.record(stream)
    torch.cuda.synchronize()
    graph_ms = a.elapsed_time(b)
    solve_ms = graph_ms / steps - density_ms
    log("graph %.1f ms: %.3f ms/step, density %.3f ms, solve %.3f ms" % (graph_ms, graph_ms / steps, density_ms,
                                                                         solve_ms))
    cell_modes = float(mesh.ncells) * mesh.nmodes
    mflops, eflops, min_bytes = plan.work()
    products = {"fp64": 1, "bf16x3": 6, "fp16x2": 3, "fp64sep": 1, "bf16x3sep": 6}[precision]
    roof = roofline(plan, phases, precision, args.workload)
    roof["solve"] = solve_bound(plan, precision, solve_ms)
    result = {"metric": METRIC, "value": cell_modes / (solve_ms * 1e-3), "unit": UNIT, "n_gpus": 1,
              "steps": steps, "warmup": args.warmup, "ms_per_step": graph_ms / steps, "higher_is_better": True,
              "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[precision], "data": "synthetic",
              "config": {"workload": args.workload, "nr": mesh.nr, "ntheta": mesh.ntheta, "nphi": mesh.nphi,
                         "lmax": mesh.lmax, "precision": precision, "hip_graph": True, "solves_per_graph": steps},
              "roofline": roof, "graph_ms": graph_ms, "density_update_ms": density_ms, "solve_ms": solve_ms,
              "solve_tflops_algorithmic": (mflops + eflops) / (solve_ms * 1e-3) / 1e12,
              "solve_tflops_executed_lower_bound": products * (mflops + eflops) / (solve_ms * 1e-3) / 1e12,
              "solve_min_hbm_gbs": min_bytes / (solve_ms * 1e-3) / 1e9,
              "plan_ms": plan_ms, "tuning": plan.tuning(), "autotuned": not args.no_tune, "tune_s": tune_s}
    # error against the FP64 GPU path every `every` steps
    if not args.no_fp64:
        p64 = mpole.Plan.from_mesh(mesh, precision="fp64", device=dev)
        errs = {}
        for k, snap in enumerate(snaps):
            t = (k + 1) * every
            gen.write(rho, t)
            ref = p64.solve(rho, ang=False, interior=False, exterior=False)["phi"]
            torch.cuda.synchronize()
            errs[t] = float((snap - ref).abs().div(ref.abs()).max())
            log("step %d: max rel err vs FP64 %.3e" % (t, errs[t]))
            del ref
        result["max_rel_err_vs_fp64_gpu_by_step"] = errs
        result["max_rel_err_vs_fp64_gpu"] = max(errs.values()) if errs else None
        del p64
    if not args.no_cpu_baseline:
        import oracle
        oracle.set_threads(host_threads())
        # bounded sample: the oracle on the 40 innermost shells of the same
        # angular mesh and lmax (merged like the full mesh), one solve
        sub = wl.large_mesh(nr=40)
        sub.shell_class, sub.class_block = wl.production_merge(40, mesh.ntheta, mesh.nphi, inner_shells=32)
        rho_s = np.ascontiguousarray(wl.radial_profile(sub)[:, None, None]
                                     * wl.rotated_angular_factor(sub, np.eye(3), coef)[None])
        ref = oracle.solve(rho=rho_s, **sub.oracle_kwargs())
        result["cpu_baseline"] = {"value": float(sub.ncells) * sub.nmodes / ref["seconds"][1], "unit": UNIT,
                                  "cores": oracle.threads(), "kind": "oracle", "cpu_model": cpu_model(),
                                  "sample": "one oracle solve of the 40 innermost shells of the same angular mesh and "
                                            "lmax (tables %.1f s excluded; solve %.1f s)" % tuple(ref["seconds"])}
    print(json.dumps(result), flush=True)


def bench_batch(args, precision):
    """64 seeded fields of uneven size and lmax solved as one batch, captured
    once in a HIP graph and replayed: the persistent launch (one launch over
    per-XCD work queues) is the measured line; the per-phase launch of the
    same batch is timed beside it and must agree bitwise."""
    import torch
    from paper_2602_02507_amd import mpole
    from paper_2602_02507_amd import workloads as wl
    dev = torch.device("cuda:0")
    meshes = wl.batch_meshes(64)
    print("bench: generating 64 densities", file=sys.stderr, flush=True)
    rho_h = wl.batch_densities(meshes)
    rho = [torch.from_numpy(r).to(dev) for r in rho_h]
    cell_modes = float(sum(m.ncells * m.nmodes for m in meshes))
    stream = torch.cuda.current_stream(dev)

    tunings, tune_info = {}, {}
    if not args.no_tune:
        from paper_2602_02507_amd import tune
        for prec in ([precision] if precision == "fp64" or args.no_fp64 else [precision, "fp64"]):
            print("bench: autotuning %s launches of the 64 fields" % prec, file=sys.stderr, flush=True)
            tunings[prec], tune_info[prec] = tune.tune_batch(meshes, prec, dev, rho=rho)
            print("bench: tuned %s in %.1f s (%d new shapes)" % (prec, tune_info[prec]["seconds"],
                                                                 tune_info[prec]["field_shapes_tuned"]),
                  file=sys.stderr, flush=True)

    def timed_batch(prec, launch="persistent"):
        batch = mpole.Batch(meshes, precision=prec, rho=rho, device=dev, tunings=tunings.get(prec), launch=launch)
        for _ in range(args.warmup):
            batch.solve()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            batch.solve()
        g.replay()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(args.steps):
            g.replay()
        b.record(stream)
        torch.cuda.synchronize()
        batch.check()
        return batch, a.elapsed_time(b) / args.steps

    fp64_ms = None
    if precision != "fp64" and not args.no_fp64:
        b64, fp64_ms = timed_batch("fp64")
        phi64 = [p.clone() for p in b64.phi]
        del b64
        torch.cuda.empty_cache()
        print("bench: fp64 batch %.3f ms" % fp64_ms, file=sys.stderr, flush=True)
    phased, phases_ms = timed_batch(precision, "phases")
    field_ph = np.array(phased.field_ms())
    print("bench: %s batch, one launch per phase: %.3f ms; field completion p50 %.3f p99 %.3f ms" % (
        precision, phases_ms, np.percentile(field_ph, 50), np.percentile(field_ph, 99)), file=sys.stderr, flush=True)
    batch, ms = timed_batch(precision)
    field = np.array(batch.field_ms())
    print("bench: %s batch, %s launch: %.3f ms; field completion p50 %.3f p99 %.3f ms%s" % (
        precision, batch.launch, ms, np.percentile(field, 50), np.percentile(field, 99),
        "" if batch.launch == "persistent" else " (" + batch.launch_note + ")"), file=sys.stderr, flush=True)
    launches_equal = all(bool(torch.equal(p, q)) for p, q in zip(batch.phi, phased.phi))
    del phased
    torch.cuda.empty_cache()
    result = {"metric": METRIC, "value": cell_modes / (ms * 1e-3), "unit": UNIT, "n_gpus": 1, "steps": args.steps,
              "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
              "vs_baseline": None, "dtype": DTYPE[precision], "data": "synthetic",
              "config": {"workload": args.workload, "fields": len(meshes), "cells": int(sum(m.ncells for m in meshes)),
                         "cell_modes": cell_modes, "precision": precision, "hip_graph": True},
              "launch": batch.launch,
              "field_ms_p50": float(np.percentile(field, 50)), "field_ms_p99": float(np.percentile(field, 99)),
              "phases_launch": {"ms_per_step": phases_ms, "field_ms_p50": float(np.percentile(field_ph, 50)),
                                "field_ms_p99": float(np.percentile(field_ph, 99)),
                                "bitwise_equal_to_persistent": launches_equal},
              "autotuned": not args.no_tune,
              "tuning_summary": _tuning_summary(tunings.get(precision)),
              "tune_s": {k: v["seconds"] for k, v in tune_info.items()}}
    if fp64_ms is not None:
        result["fp64_ms_per_step"] = fp64_ms
        result["speedup_vs_fp64"] = fp64_ms / ms
        result["max_rel_err_vs_fp64_gpu"] = max(float((p - q).abs().div(q.abs()).max())
                                                for p, q in zip(batch.phi, phi64))
    if not (args.no_cpu_baseline and args.no_check):
        import oracle
        oracle.set_threads(host_threads())
        # bounded sample: the oracle on the four smallest fields
        order = np.argsort([m.ncells * m.nmodes for m in meshes])[:4]
        t_solve, cm, err = 0.0, 0.0, 0.0
        for f in order:
            ref = oracle.solve(rho=rho_h[f], **meshes[f].oracle_kwargs())
            t_solve += ref["seconds"][1]
            cm += meshes[f].ncells * meshes[f].nmodes
            got = batch.phi[f].cpu().numpy()
            err = max(err, float(np.max(np.abs(got - ref["phi"]) / np.abs(ref["phi"]))))
        if not args.no_cpu_baseline:
            result["cpu_baseline"] = {"value": cm / t_solve, "unit": UNIT, "cores": oracle.threads(), "kind": "oracle",
                                      "cpu_model": cpu_model(),
                                      "sample": "oracle solves of the 4 smallest fields (%.2e cell-modes, %.2f s)"
                                                % (cm, t_solve)}
        if not args.no_check:
            result["max_rel_err_vs_oracle_sampled_fields"] = err
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
