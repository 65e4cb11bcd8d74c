"""Time loop of a problem to an exact final time: whole steps (`esvdw_step`) replayed from a HIP
graph in blocks, so that small grids are not bound by per-launch latency, then single steps,
and the last two steps of equal fixed length so the run ends on t_end.

A block is `block` steps captured once into a graph; each captured step writes its dt to its
own slot of a device array, which the host reads after every replay to advance t.  Blocks run
while the remaining time exceeds twice (block + 2) last steps (room for dt to grow within a block);
then single steps run until two fixed steps of half the remaining time finish the run."""
from .esvdw import Context


def advance_to(torch, ctx, p, JU, J, x, moving, t_end, block=20, log=None, stream=None):
    """Returns dict(steps, t, gpu_ms, flags, graph_steps)."""
    f64 = dict(dtype=torch.float64, device=JU.device)
    st = stream or torch.cuda.current_stream()
    dts = torch.zeros(block, **f64)
    dt1 = torch.zeros(1, **f64)
    mv = 1 if moving else 0
    t, steps, gpu_ms, last_dt, graph_steps = 0.0, 0, 0.0, 0.0, 0
    ev = lambda: torch.cuda.Event(enable_timing=True)

    def timed(fn):
        e0, e1 = ev(), ev()
        e0.record(st)
        fn()
        e1.record(st)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    # one direct step first: it sets last_dt and warms the kernels before capture
    gpu_ms += timed(lambda: ctx.step(JU, J, x, mv, dt1, st))
    last_dt = float(dt1.item())
    t += last_dt
    steps += 1
    graph = None
    while block > 1 and t_end - t > 2.0 * (block + 2) * last_dt:
        if graph is None:
            side = torch.cuda.Stream()
            side.wait_stream(st)
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.stream(side):
                with torch.cuda.graph(graph, stream=side):
                    for k in range(block):
                        ctx.step(JU, J, x, mv, dts[k:k + 1], side)
            torch.cuda.synchronize()
            # capture records without running: replay below performs the steps
        cur = torch.cuda.current_stream()
        e0, e1 = ev(), ev()
        e0.record(cur)
        graph.replay()
        e1.record(cur)
        torch.cuda.synchronize()
        gpu_ms += e0.elapsed_time(e1)
        d = dts.cpu().tolist()
        t += sum(d)
        last_dt = d[-1]
        steps += block
        graph_steps += block
        if log and steps % (25 * block) < block:
            log("step %d t %.5f / %.5f" % (steps, t, t_end))
    tail = None
    cur_ctx = ctx
    while t < t_end * (1.0 - 1e-14):
        if tail is None and t_end - t < 2.0 * last_dt:
            tail = Context(dict(p, dt_fixed=0.5 * (t_end - t)))
            cur_ctx = tail
        gpu_ms += timed(lambda: cur_ctx.step(JU, J, x, mv, dt1, st))
        last_dt = float(dt1.item())
        t += last_dt
        steps += 1
    flags = ctx.status() | (tail.status() if tail is not None else 0)
    return dict(steps=steps, t=t, gpu_ms=gpu_ms, flags=flags, graph_steps=graph_steps)
