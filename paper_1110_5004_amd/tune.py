"""Launch-shape autotuner.

Times every compiled tile variant of the step on the cases of a live
Simulation, with HIP events on the stream the library launches on, and keeps
the fastest.  For D2Q9 it also times a few persistent grid sizes (workgroups
walking the tile list) of the variants within 5 % of the best one-workgroup-
per-tile launch; the D3Q19 kernels always launch one workgroup per tile.
Every measurement replays the captured step graph: the graph is built before
the timed window and a whole number of graph replays is timed.  Choices are
cached in a JSON file keyed by lattice, storage, model switch, a node-count
bucket and a hash of the built library, so a later Simulation of the same
kind (and of the same kernels) starts from the tuned shape.  Tuning changes
no result: every variant computes each node with the same arithmetic.
"""
import hashlib
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
    return f"lat{p['lattice']}_{st}_rf{rf}_n{bucket}_c{len(sim.dims)}_v{nv}_{_lib_hash()}"


_LIB_HASH = None


def _lib_hash():
    """Short hash of the built library: winners measured on other kernels
    are not reused."""
    global _LIB_HASH
    if _LIB_HASH is None:
        h = hashlib.sha256()
        with open(B.LIB_PATH, "rb") as f:
            for blk in iter(lambda: f.read(1 << 20), b""):
                h.update(blk)
        _LIB_HASH = h.hexdigest()[:12]
    return _LIB_HASH


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
    """Seconds per step of one launch shape (HIP events on the library's
    stream).  The graph is captured first and the timed window starts at an
    even step, so it holds whole graph replays only: steps is rounded up to a
    multiple of graph_steps."""
    torch = sim.torch
    sim.set_launch(variant, grid, graph_steps)
    sim.prepare()
    if graph_steps >= 2:
        steps = graph_steps * max(1, -(-steps // graph_steps))
    sim.step(max(2, graph_steps) + (sim.time & 1))  # warm the caches; even parity
    stream = torch.cuda.current_stream(sim.device)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    torch.cuda.synchronize(sim.device)
    return e0.elapsed_time(e1) / 1e3 / steps


def persistent_grids(sim):
    """Persistent grid sizes (workgroups walking the tile list) worth timing:
    one, two and four workgroups per CU of the 256-CU device (D2Q9 only;
    workgroups beyond the tile count find no tile and exit)."""
    if sim.params[0]["lattice"] != B.D2Q9:
        return ()
    return (256, 512, 1024)


def tune(sim, steps=200, graph_steps=16, grids=None, use_cache=True, verbose=False):
    """Pick the fastest (variant, grid) for sim, apply it, return the record.

    grids: persistent grid sizes to try besides one workgroup per tile (0);
    None = persistent_grids(sim), timed on the variants within 5 % of the best
    one-workgroup-per-tile time.  The simulation advances while it is timed;
    callers that need a given time level should tune a copy or checkpoint
    first (lbm_get_state)."""
    cache = load_cache() if use_cache else {}
    key = _key(sim)
    if use_cache and key in cache:
        rec = cache[key]
        sim.set_launch(rec["variant"], rec["grid"], rec["graph_steps"])
        return dict(rec, cached=True)
    results = []
    shapes = B.variants(sim.params[0]["lattice"])
    for v, shape in enumerate(shapes):
        t = time_launch(sim, v, 0, graph_steps, steps)
        results.append((t, v, 0))
        if verbose:
            print(f"tune {key}: variant {v} {shape} grid 0: {t * 1e6:.2f} us/step", flush=True)
    best = min(results)[0]
    near = [v for t, v, _ in results if t <= 1.05 * best]
    for g in (persistent_grids(sim) if grids is None else grids):
        if g <= 0:
            continue
        for v in near:
            t = time_launch(sim, v, g, graph_steps, steps)
            results.append((t, v, g))
            if verbose:
                print(f"tune {key}: variant {v} {shapes[v]} grid {g}: {t * 1e6:.2f} us/step",
                      flush=True)
    t, v, g = min(results)
    rec = dict(variant=v, grid=g, graph_steps=graph_steps, us_per_step=t * 1e6,
               all=[dict(variant=vv, grid=gg, us_per_step=tt * 1e6) for tt, vv, gg in results])
    sim.set_launch(v, g, graph_steps)
    if use_cache:
        cache[key] = rec
        save_cache(cache)
    return dict(rec, cached=False)
