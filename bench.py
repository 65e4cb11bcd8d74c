"""Throughput benchmark of the entropy-stable adaptive moving-mesh step on one MI355X.

Workload: 2D van der Waals four-quadrant Riemann problem on [0,1]^2, 1024 x 1024 nodes,
reduced units (R = 8/3, c_v = R/0.0125, a = 3, b = 1/3), outflow boundaries, quadrant
states drawn with seed 0; one step = mesh redistribution (monitor with rho and G,
5 filter passes, mu = 10 Jacobi sweeps, limiter, CFL 0.4) + three SSP-RK3 stages of the
sixth-order EC + MR-WENO5 entropy-stable RHS on the moving mesh.  The step is captured in a
HIP graph and replayed; inputs are resident in HBM.

Prints one JSON line.  value = node-stages per second = nodes * 3 * steps / time.
"""
import argparse
import json
import math
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
# algorithmic HBM bytes of one flux-kernel interface: one read of a node's 17 fields
# (rho, v1, v2, T, p, 1/T, g, 4 entropy variables, 4 metrics, 2 grid-speed metrics) and one
# write of the 5 flux values
BYTES_PER_IFACE_2D = 17 * 8 + 5 * 8
# the copy kernel of esvdw_bench_kernel(6): 2 (dim + 3) N doubles, read once and written once
COPY_DOUBLES_2D = lambda n: 5 * n * n
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


def cpu_baseline(size, seed):
    """The oracle on the host: one moving-mesh step of the same problem (bounded sample)."""
    import numpy as np
    import oracle
    from paper_2407_05568_amd import synth
    p = synth.problem(2, [size, size], bc="outflow")
    o = oracle.Oracle(p)
    x = o.uniform_mesh()
    J = o.jacobian(x)
    JU = o.init_state(synth.quadrants_2d(p, synth.quadrant_states(p, seed)), J)
    t0 = time.perf_counter()
    o.step(JU, J, x, moving=True)
    el = time.perf_counter() - t0
    return {"value": size * size * 3 / el, "unit": "node-stages/s", "cores": 1, "kind": "oracle",
            "sample": "one moving-mesh step of the same 2D four-quadrant problem at %dx%d (%.1f s, single thread)"
                      % (size, size, el)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--size", type=int, default=1024)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-size", type=int, default=1024)
    ap.add_argument("--kernel-reps", type=int, default=20)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only (the path shards by spatial domain "
              "decomposition, see the design notes); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2407_05568_amd import synth
    from paper_2407_05568_amd.esvdw import Context

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    n = args.size
    p = synth.problem(2, [n, n], bc="outflow")
    ctx = Context(p)
    states = synth.quadrant_states(p, args.seed)
    prim = torch.from_numpy(synth.quadrants_2d(p, states)).to(dev)
    x = torch.empty((2, n, n), dtype=torch.float64, device=dev)
    J = torch.empty((n, n), dtype=torch.float64, device=dev)
    JU = torch.empty((4, n, n), dtype=torch.float64, device=dev)
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
    node_stages = n * n * 3 * args.steps
    value = node_stages / (ms / 1e3)
    print("timed %d steps: %.3f ms/step, status %d" % (args.steps, ms_per_step, status), file=sys.stderr, flush=True)

    # dominant kernel: the interface-flux kernel, timed live on the same stream
    k0, k1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = args.kernel_reps
    k0.record(stream)
    ctx.bench_kernel(1, reps, stream)
    ctx.bench_kernel(2, reps, stream)
    k1.record(stream)
    torch.cuda.synchronize()
    t_launch = k0.elapsed_time(k1) / 1e3 / (2 * reps)
    # plain copy of a known size (reads and writes COPY_BYTES each): the calibration kernel of
    # the hardware byte counters
    ctx.bench_kernel(6, 2, stream)
    torch.cuda.synchronize()
    nif = (n + 1) * n
    achieved = FLOPS_PER_IFACE_2D * nif / t_launch
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64, "traffic": measured_traffic(n),
                "kernel": "k_flux (2D interface flux, %d interfaces per launch)" % nif,
                "avg_launch_ms": t_launch * 1e3,
                "algorithmic_bytes_GBps": BYTES_PER_IFACE_2D * nif / t_launch / 1e9}

    cpu = None
    if not args.no_cpu:
        print("cpu baseline ...", file=sys.stderr, flush=True)
        cpu = cpu_baseline(args.cpu_size, args.seed)

    out = {
        "metric": "FP64 cell-stage updates/s (2D 1024² moving mesh)",
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
        "config": {"workload": "2D vdW four-quadrant Riemann problem, %dx%d adaptive moving mesh, seed %d" % (
            n, n, args.seed), "scheme": "6th-order EC flux + MR-WENO5 ES dissipation, SSP-RK3, CFL 0.4",
                   "mesh": "vdW monitor (rho, G), 5 filter passes, mu=10 Jacobi sweeps", "graph": graph is not None,
                   "status_flags": status},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
