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

# algorithmic FP64 operation counts (each +, -, *, /, sqrt, log, log1p, min, max, abs = 1)
# per 2D interface of the flux kernel: the two-point EC fluxes of the pairs the interface
# owns (3 pairs of ~150 operations, plus the alpha combination of its 6 pair fluxes) and
# the dissipation (averaged state and eigen-system ~130, W on the 6-node stencil ~150,
# rounding scale of W ~60, 8 MR-WENO5 reconstructions of ~87, sign matrix and projection
# back ~60).
FLOPS_PER_IFACE_2D = 3 * 150 + 60 + 130 + 150 + 60 + 8 * 87 + 60
# per 2D node-stage: two interfaces, the node kernel (~100) and the update (~20)
FLOPS_PER_NODE_STAGE_2D = 2 * FLOPS_PER_IFACE_2D + 120
# 3D interface (estimate on the same counting rules): 3 pair fluxes of ~180, combination ~70,
# averaged state and 3D eigen-system ~160, W on 6 nodes ~210, rounding scale ~80, 10 MR-WENO5
# reconstructions of ~87, projection ~80
FLOPS_PER_IFACE_3D = 3 * 180 + 70 + 160 + 210 + 80 + 10 * 87 + 80
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


def measured_traffic(n):
    """HBM bytes per k_flux launch from the committed counter summary (FETCH_SIZE + WRITE_SIZE,
    each scaled by the copy kernel's reading), if it was taken on the current kernel source
    at this size; else None."""
    path = os.path.join(ROOT, "profiles", "k_flux_2d_1024_counters.md")
    try:
        with open(path) as f:
            txt = f.read()
        blob = txt.split("```json")[1].split("```")[0]
        d = json.loads(blob)
    except (OSError, IndexError, ValueError):
        return None
    if d.get("source_hash") != kernel_source_hash() or d.get("size") != n:
        return None
    return d.get("traffic_bytes_per_launch")


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


def cpu_baseline(workload, size, seed, steps):
    """The oracle on the host: `steps` moving-mesh steps of the same problem (bounded sample)."""
    import oracle
    p = make_problem(workload, size)
    o = oracle.Oracle(p)
    x = o.uniform_mesh()
    J = o.jacobian(x)
    JU = o.init_state(initial_prim(workload, p, seed), J)
    t0 = time.perf_counter()
    for _ in range(steps):
        JU, J, x, _ = o.step(JU, J, x, moving=True)
    el = time.perf_counter() - t0
    nodes = size ** p["dim"]
    return {"value": nodes * 3 * steps / el, "unit": "node-stages/s", "cores": 1, "kind": "oracle",
            "sample": "%d moving-mesh step(s) of the same %s problem at %s nodes (%.1f s, single thread)"
                      % (steps, workload, "x".join([str(size)] * p["dim"]), el)}


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

    cpu = None
    if not args.no_cpu:
        print("cpu baseline ...", file=sys.stderr, flush=True)
        cpu = cpu_baseline(args.workload, args.cpu_size or (80 if three else 1024), args.seed, 1 if three else 2)

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
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
