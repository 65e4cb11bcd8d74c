"""Throughput benchmark of the entropy-stable adaptive moving-mesh step on one MI355X.

Default workload (--workload 2d-quadrants): 2D van der Waals four-quadrant Riemann problem on
[0,1]^2, 1024 x 1024 nodes, reduced units (R = 8/3, c_v = R/0.0125, a = 3, b = 1/3), outflow
boundaries, quadrant states drawn with seed 0; one step = mesh redistribution (monitor with rho
and G, 5 filter passes, mu = 10 Jacobi sweeps, limiter, CFL 0.4) + three SSP-RK3 stages of the
sixth-order EC + MR-WENO5 entropy-stable RHS on the moving mesh.

--workload 3d-smooth: 3D periodic smooth vdW flow on [0,1]^3 at 192^3 (rho = 1 + 0.2 sum of
four random-phase sine modes with |k|_inf <= 4, v = (0.3, 0.2, 0.1), p = 1.2), linear weights
1/3 each, CFL 0.3, moving mesh driven by the density-gradient monitor (alpha = 20, 5 filter
passes, mu = 10 sweeps).

The step is captured in a HIP graph and replayed; inputs are resident in HBM.
Prints one JSON line.  value = node-stages per second = nodes * 3 * steps / time.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic FP64 operation counts (each +, -, *, /, sqrt, log, min, max, abs = 1), from the
# per-node-stage budget of the scheme in 2D: about 3.7 kflop per node and RK stage, of which
# about 0.3 k is node thermodynamics and the update and 3.4 k the interface fluxes (two-point EC
# pair fluxes ~1.0 k, MR-WENO reconstructions ~1.76 k, projections ~0.38 k, averaged state and
# eigen-system ~0.26 k), i.e. 1.7 k per interface (a node-stage owns one interface per direction).
FLOPS_PER_IFACE_2D = 1700
# 3D: about 7.7 kflop per node-stage, ~0.3 k outside the fluxes, over three interfaces
FLOPS_PER_IFACE_3D = 2470
# algorithmic HBM bytes of one flux-kernel interface: one read of a node's 17 fields
# (rho, v1, v2, T, p, 1/T, g, 4 entropy variables, 4 metrics, 2 grid-speed metrics) and one
# write of the 5 flux values
BYTES_PER_IFACE_2D = 17 * 8 + 5 * 8
PEAK_FP64 = 78.6e12  # MI355X FP64 vector: 256 CU x 2.4 GHz x 128 FLOP/clk
PEAK_HBM = 8.0e12


def kernel_source_hash():
    """Hash of the sources the flux kernel is built from (the counters are void once they change)."""
    import hashlib
    h = hashlib.sha256()
    for f in ("rhs.hip", "scheme.h", "common.h"):
        with open(os.path.join(ROOT, "paper_2407_05568_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profile_record(name, n):
    """The machine-readable block of a committed rocprofv3 summary under profiles/, if it was
    taken on the current kernel sources at this size; else None."""
    path = os.path.join(ROOT, "profiles", name)
    try:
        with open(path) as f:
            txt = f.read()
        d = json.loads(txt.split("```json")[1].split("```")[0])
    except (OSError, IndexError, ValueError):
        return None
    if d.get("source_hash") != kernel_source_hash() or d.get("size") != n:
        return None
    return d


def measured_traffic(n):
    """HBM bytes per k_flux launch from the committed counter summary (FETCH_SIZE + WRITE_SIZE,
    each scaled by the copy kernel's reading); None unless taken on the current sources."""
    d = profile_record("kernels_2d_1024_counters.md", n)
    return None if d is None else d.get("traffic_bytes_per_launch")


def in_step_flux_us(n):
    """Average k_flux duration inside graph-replayed steps, from the committed kernel trace of
    the step (rocprofv3 --kernel-trace); None unless taken on the current sources."""
    d = profile_record("kernels_2d_1024_moving_step.md", n)
    return None if d is None else d.get("k_flux_in_step_us")


def make_problem(workload, n):
    from paper_2407_05568_amd import synth
    if workload == "3d-smooth":
        return synth.problem(3, [n, n, n], bc="periodic", weno_lin=[1 / 3, 1 / 3, 1 / 3], kappa=1,
                             mon_var=["rho"], alpha=[20.0, 0.0, 0.0])
    return synth.problem(2, [n, n], bc="outflow")


def initial_prim(workload, p, seed):
    from paper_2407_05568_amd import synth
    if workload == "3d-smooth":
        return synth.smooth_3d(p, seed)
    return synth.quadrants_2d(p, synth.quadrant_states(p, seed))


def cpu_baseline(workload, size, seed, steps, steps_mt):
    """The oracle on the host's cores, on a bounded sample of the same workload: `steps_mt`
    moving-mesh steps with its OpenMP build on every core this process may run on
    (os.sched_getaffinity), and `steps` with the single-thread build (the one the parity tests
    use); both start from the same initial data.  The OpenMP build is the same source with its
    outer node loops split across threads (identical results)."""
    import oracle
    p = make_problem(workload, size)
    prim = initial_prim(workload, p, seed)
    nodes = size ** p["dim"]
    out = {}
    cores = len(os.sched_getaffinity(0))
    for mt in (True, False):
        o = oracle.Oracle(p, omp=mt)
        threads = o.L.orc_threads(cores if mt else 1)
        x = o.uniform_mesh()
        J = o.jacobian(x)
        JU = o.init_state(prim, J)
        n = steps_mt if mt else steps
        t0 = time.perf_counter()
        for _ in range(n):
            JU, J, x, _ = o.step(JU, J, x, moving=True)
        el = time.perf_counter() - t0
        out[mt] = dict(value=nodes * 3 * n / el, unit="node-stages/s", cores=threads, seconds=el, steps=n)
    grid = "x".join([str(size)] * p["dim"])
    res = {"value": out[True]["value"], "unit": "node-stages/s", "cores": out[True]["cores"], "kind": "oracle",
           "sample": "%d moving-mesh step(s) of the same %s problem at %s nodes, OpenMP build on %d threads "
                     "(%.1f s)" % (out[True]["steps"], workload, grid, out[True]["cores"], out[True]["seconds"]),
           "single_thread": {"value": out[False]["value"], "unit": "node-stages/s", "cores": 1,
                             "sample": "%d step(s), %.1f s" % (out[False]["steps"], out[False]["seconds"])}}
    return res


WARMSTART = os.path.join(ROOT, "paper_2407_05568_amd", "mlp_warmstart_1024.npz")


def learned_speedup(torch, n=1024, seed=2, step=5, tol=1e-8):
    """The learned warm start against the plain iteration on one frame of a held-out run (the
    network's weights were trained on other seeds by `python -m paper_2407_05568_amd.learned
    --size 1024 --save ...`): the redistribution of the state after `step` steps of the method
    solved to the residual tol by red-black SOR from x^n (plain) and from x^n + the network's
    displacement (features + inference + 8 Gauss-Seidel sweeps + SOR), and, for reference, from
    the previous step's converged mesh (not learned); each timed twice after one untimed round,
    the means kept.  value = plain time / warm time."""
    from paper_2407_05568_amd import learned, synth
    P, meta = learned.load_params(WARMSTART)
    Pd = torch.from_numpy(P).cuda()
    p = synth.problem(2, [n, n], bc="outflow")
    run = learned.Run(torch, p, synth.quadrants_2d(p, synth.quadrant_states(p, seed)), tol)
    sor = learned.SorSolver(torch, run)
    run.advance(step - 1)
    sor.solve(1e-10)
    xprev = sor.x.clone()
    run.advance(1)
    shape = (n, n)
    feat = torch.empty((2,) + shape, dtype=torch.float32, device="cuda")
    warm = torch.empty((2,) + shape, dtype=torch.float64, device="cuda")
    times = {"inf": [], "w": [], "p": [], "q": []}
    for rep in range(3):  # the first round warms every kernel and is not counted
        ms_inf = learned.warm_start(torch, run, Pd, feat, warm)
        sw_w, res_w, ms_w = sor.solve(tol, warm=warm, presmooth=8)
        sw_p, res_p, ms_p = sor.solve(tol)
        sw_q, res_q, ms_q = sor.solve(tol, start=xprev)
        if rep:
            for k, v in (("inf", ms_inf), ("w", ms_w), ("p", ms_p), ("q", ms_q)):
                times[k].append(v)
    ms_inf, ms_w, ms_p, ms_q = (sum(times[k]) / len(times[k]) for k in ("inf", "w", "p", "q"))
    return {"value": ms_p / (ms_w + ms_inf), "unit": "x (plain / warm-started redistribution time)",
            "plain_ms": ms_p, "warm_ms": ms_w + ms_inf, "inference_ms": ms_inf, "plain_sweeps": sw_p,
            "warm_sweeps": sw_w, "final_residual": max(res_p, res_w), "tolerance": tol,
            "previous_mesh_speedup": ms_p / ms_q,
            "sample": "seed %d (held out), state after %d steps of the %dx%d quadrant run; weights trained on "
                      "seeds %s" % (seed, step, n, n, meta.get("train_seeds"))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["2d-quadrants", "3d-smooth"], default="2d-quadrants")
    ap.add_argument("--size", type=int, default=None)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-size", type=int, default=None)
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--no-learned", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the solver runs on one GPU (several would split the grid into slabs with halo "
              "exchanges, which is not implemented); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2407_05568_amd.esvdw import Context

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    three = args.workload == "3d-smooth"
    n = args.size or (192 if three else 1024)
    p = make_problem(args.workload, n)
    d = p["dim"]
    ctx = Context(p)
    prim = torch.from_numpy(initial_prim(args.workload, p, args.seed)).to(dev)
    shape = (n,) * d
    x = torch.empty((d,) + shape, dtype=torch.float64, device=dev)
    J = torch.empty(shape, dtype=torch.float64, device=dev)
    JU = torch.empty((d + 2,) + shape, dtype=torch.float64, device=dev)
    dt = torch.zeros(1, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    ctx.init_mesh(x, J, 1, stream)
    ctx.init_state(prim, J, JU, stream)
    for _ in range(args.warmup):
        ctx.step(JU, J, x, 1, dt, stream)
    torch.cuda.synchronize()
    print("warmup done", file=sys.stderr, flush=True)

    graph = None
    if not args.no_graph:
        try:
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                ctx.step(JU, J, x, 1, dt)
            graph = g
        except Exception as e:  # capture unsupported: time direct launches
            print("graph capture failed (%s); timing direct launches" % e, file=sys.stderr)
            graph = None
    torch.cuda.synchronize()

    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        if graph is not None:
            graph.replay()
        else:
            ctx.step(JU, J, x, 1, dt, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    status = ctx.status()
    ms_per_step = ms / args.steps
    nodes = n ** d
    node_stages = nodes * 3 * args.steps
    value = node_stages / (ms / 1e3)
    print("timed %d steps: %.3f ms/step, status %d" % (args.steps, ms_per_step, status), file=sys.stderr, flush=True)

    # the same step on the current (fixed) mesh: CFL + three RK stages, no redistribution
    # (separate state copy; the timed run above is unaffected)
    JUf, Jf, xf = JU.clone(), J.clone(), x.clone()
    dtf = torch.zeros(1, dtype=torch.float64, device=dev)
    ctx.step(JUf, Jf, xf, 0, dtf, stream)
    torch.cuda.synchronize()
    f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    f0.record(stream)
    for _ in range(args.steps):
        ctx.step(JUf, Jf, xf, 0, dtf, stream)
    f1.record(stream)
    torch.cuda.synchronize()
    ms_fixed = f0.elapsed_time(f1) / args.steps
    rhs_only = {"ms_per_step": ms_fixed, "node_stages_per_s": nodes * 3 / (ms_fixed / 1e3),
                "what": "CFL + three RK stages on the current mesh, no redistribution (direct launches)"}
    del JUf, Jf, xf

    # dominant kernel: the interface-flux kernel, timed live on the same stream
    k0, k1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = args.kernel_reps
    k0.record(stream)
    for k in range(d):
        ctx.bench_kernel(k + 1, reps, stream)
    k1.record(stream)
    torch.cuda.synchronize()
    t_launch = k0.elapsed_time(k1) / 1e3 / (d * reps)
    # plain copy of a known size (reads and writes COPY_BYTES each): the calibration kernel of
    # the hardware byte counters
    ctx.bench_kernel(6, 2, stream)
    torch.cuda.synchronize()
    nif = (n + 1) * n ** (d - 1)
    achieved = (FLOPS_PER_IFACE_3D if three else FLOPS_PER_IFACE_2D) * nif / t_launch
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64, "traffic": None if three else measured_traffic(n),
                "kernel": "k_flux (%dD interface flux, %d interfaces per launch)" % (d, nif),
                "avg_launch_ms": t_launch * 1e3}
    if not three:
        roofline["algorithmic_bytes_GBps"] = BYTES_PER_IFACE_2D * nif / t_launch / 1e9
        t_in = in_step_flux_us(n)
        roofline["in_step_launch_ms"] = None if t_in is None else t_in / 1e3
        roofline["frac_in_step"] = None if t_in is None else FLOPS_PER_IFACE_2D * nif / (t_in * 1e-6) / PEAK_FP64
    roofline["flops_per_interface"] = FLOPS_PER_IFACE_3D if three else FLOPS_PER_IFACE_2D

    learned = None
    if not three and not args.no_learned and n == 1024:
        print("learned warm start ...", file=sys.stderr, flush=True)
        learned = learned_speedup(torch)

    cpu = None
    if not args.no_cpu:
        print("cpu baseline ...", file=sys.stderr, flush=True)
        cpu = cpu_baseline(args.workload, args.cpu_size or (80 if three else 1024), args.seed, 1, 2 if three else 3)

    if three:
        metric = "FP64 cell-stage updates/s (3D %d³ moving mesh)" % n
        cfg = {"workload": "3D periodic smooth vdW flow, %d^3 adaptive moving mesh, seed %d" % (n, args.seed),
               "scheme": "6th-order EC flux + MR-WENO5 ES dissipation (linear weights 1/3), SSP-RK3, CFL 0.3",
               "mesh": "density-gradient monitor (alpha 20), 5 filter passes, mu=10 Jacobi sweeps"}
    else:
        metric = "FP64 cell-stage updates/s (2D 1024² moving mesh)"
        cfg = {"workload": "2D vdW four-quadrant Riemann problem, %dx%d adaptive moving mesh, seed %d" % (
            n, n, args.seed), "scheme": "6th-order EC flux + MR-WENO5 ES dissipation, SSP-RK3, CFL 0.4",
               "mesh": "vdW monitor (rho, G), 5 filter passes, mu=10 Jacobi sweeps"}
    cfg.update({"graph": graph is not None, "status_flags": status})
    out = {
        "metric": metric,
        "value": value,
        "unit": "node-stages/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": cfg,
        "rhs_only": rhs_only,
        "roofline": roofline,
        "learned_speedup": learned,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
