"""Launch-shape autotuner.

Times every compiled tile variant (and a few persistent grid sizes) of the
fused step on the cases of a live Simulation, with HIP events on the stream
the library launches on, and keeps the fastest.  Choices are cached in a JSON
file keyed by lattice, storage, model switch and a node-count bucket, so a
later Simulation of the same kind starts from the tuned shape.  Tuning changes
no result: every variant computes each node with the same arithmetic.
"""
import json
import math
import os

from . import binding as B

CACHE = os.environ.get("LBM_TUNE_CACHE",
                       os.path.join(os.path.dirname(os.path.abspath(__file__)), "_build",
                                    "tune_cache.json"))


def _key(sim):
    p = sim.params[0]
    nodes = sum(int(d[0] * d[1] * d[2]) for d in sim.dims)
    bucket = 2 ** int(round(math.log2(max(nodes, 1))))
    rf = max(int(q["remove_fa"]) for q in sim.params)
    st = sim.storage_name
    # the number of compiled variants: a library with another variant table
    # does not reuse the winner measured on this one
    nv = len(B.variants(p["lattice"]))
    return f"lat{p['lattice']}_{st}_rf{rf}_n{bucket}_c{len(sim.dims)}_v{nv}"


def load_cache(path=CACHE):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(cache, path=CACHE):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_launch(sim, variant, grid, graph_steps, steps):
    """Seconds per step of one launch shape (HIP events on the library's stream)."""
    torch = sim.torch
    sim.set_launch(variant, grid, graph_steps)
    sim.step(max(2, graph_steps))            # warm: capture the graph, fill caches
    stream = torch.cuda.current_stream(sim.device)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    torch.cuda.synchronize(sim.device)
    return e0.elapsed_time(e1) / 1e3 / steps


def tune(sim, steps=200, graph_steps=16, grids=(0,), use_cache=True, verbose=False):
    """Pick the fastest (variant, grid) for sim, apply it, return the record.

    The simulation advances while it is timed; callers that need a given time
    level should tune a copy or checkpoint first (lbm_get_state)."""
    cache = load_cache() if use_cache else {}
    key = _key(sim)
    if use_cache and key in cache:
        rec = cache[key]
        sim.set_launch(rec["variant"], rec["grid"], rec["graph_steps"])
        return dict(rec, cached=True)
    results = []
    for v, shape in enumerate(B.variants(sim.params[0]["lattice"])):
        for g in grids:
            t = time_launch(sim, v, g, graph_steps, steps)
            results.append((t, v, g))
            if verbose:
                print(f"tune {key}: variant {v} {shape} grid {g}: {t * 1e6:.2f} us/step",
                      flush=True)
    t, v, g = min(results)
    rec = dict(variant=v, grid=g, graph_steps=graph_steps, us_per_step=t * 1e6,
               all=[dict(variant=vv, grid=gg, us_per_step=tt * 1e6) for tt, vv, gg in results])
    sim.set_launch(v, g, graph_steps)
    if use_cache:
        cache[key] = rec
        save_cache(cache)
    return dict(rec, cached=False)
