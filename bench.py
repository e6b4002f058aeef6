"""Benchmark of the fused phase-field LBM step on one MI355X.

Workload: droplet splash on a thin film, 1024 x 512 D2Q9, periodic in x,
bounce-back walls in y, FP32 populations, corrected model (the whole path
including the lap mu stencil of the -F_a correction).  A step is one lattice
time step of the whole grid; the default K = 20000 steps is the workload's
length.  Inputs are resident in HBM before timing starts.

Prints one JSON line: MLUPS (lattice updates per second / 1e6), the roofline
of the fused step kernel (algorithmic bytes 148 B per lattice update in FP32:
18 float populations plus the 2-byte low part of f_0, read once and written
once), the FP64 CPU oracle timed on a
bounded sample of the same workload, and the same measurements for FP16
storage (76 B per update), the original model and the correction with F_a's
rate taken from the data (156 B per update in FP32).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_LU = {"fp32": 148.0, "fp16": 76.0, "bf16": 76.0}
# the correction from data (remove_fa = 2) also reads and writes one float of
# phi per node
PHI_PLANE_BYTES = 8.0
BYTES_PER_LU_3D = {"fp32": 308.0, "fp16": 156.0, "bf16": 156.0}
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "traffic.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--storage", default="fp32")
    ap.add_argument("--remove-fa", type=int, default=1, choices=[0, 1, 2])
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="skip the FP16 / original-model legs")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--workload", default="splash1024x512",
                    choices=["splash1024x512", "droplet4096", "splash3d", "fa_diagnostics"],
                    help="splash1024x512 (the benchmark), droplet4096 (profiling of "
                         "the HBM-bound regime), splash3d (the D3Q19 step alone) or "
                         "fa_diagnostics (the two F_a diagnostics alone)")
    ap.add_argument("--variant", type=int, default=-1,
                    help="tile variant; -1 = autotuned")
    return ap.parse_args()


def time_gpu(torch, sim, steps, warmup):
    sim.step(warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3


def make_case(W, workload, remove_fa):
    if workload == "droplet4096":
        return W.big_droplet(remove_fa=remove_fa)
    return W.splash_2d(remove_fa=remove_fa)


def leg(torch, W, hip, storage, remove_fa, steps, warmup, workload="splash1024x512",
        variant=-1):
    from paper_1110_5004_amd import tune
    case = make_case(W, workload, remove_fa)
    sim = hip.Simulation([case], storage=storage)
    if variant >= 0:
        sim.set_launch(variant, 0, 16)
    else:
        # pick the launch shape on a scratch copy, so that the timed run starts
        # from the initial state
        probe = hip.Simulation([case], storage=storage)
        rec = tune.tune(probe, steps=100 if case.n < 4e6 else 10)
        probe.close()
        sim.set_launch(rec["variant"], rec["grid"], rec["graph_steps"])
    t = time_gpu(torch, sim, steps, warmup)
    d = sim.diagnostics()
    variant_used = sim.get_launch()[0]
    n = case.n
    mlups = n * steps / t / 1e6
    sim.close()
    return dict(mlups=mlups, seconds=t, ms_per_step=1e3 * t / steps, nodes=n,
                mass_drift_rel=d["mass_drift_rel"], nonfinite=int(d["nonfinite"]),
                umax=d["umax"], variant=variant_used)


def kernel_3d(hip, variant, remove_fa):
    """Name of the D3Q19 step a variant launches: the fused step (an x-y tile
    marching up a z chunk of 16 or more planes; k3_slab2, one plane shorter,
    for the original model) or the three-kernel step."""
    if hip.variants(hip.D3Q19)[variant][2] >= 16:
        if remove_fa == 0:
            return "k3_slab2 (fused D3Q19 step without the Eq. 5 term)"
        return "k3_slab (fused D3Q19 step)"
    return "k3_pull + k3_fields_t + k3_collide"


def leg_3d(torch, W, hip, storage, remove_fa, steps=100, warmup=10, variant=-1):
    """D3Q19 splash 256x256x128 (periodic x, y, walls z); variant -1: autotuned."""
    from paper_1110_5004_amd import tune
    case = W.splash_3d(remove_fa=remove_fa)
    if variant >= 0:
        rec = dict(variant=variant, grid=0, graph_steps=16)
    else:
        probe = hip.Simulation([case], storage=storage)
        rec = tune.tune(probe, steps=10)
        probe.close()
    sim = hip.Simulation([case], storage=storage)
    sim.set_launch(rec["variant"], rec["grid"], rec["graph_steps"])
    t = time_gpu(torch, sim, steps, warmup)
    d = sim.diagnostics()
    variant = sim.get_launch()[0]
    sim.close()
    mlups = case.n * steps / t / 1e6
    # the correction from data also reads phi^(n-1) and writes phi: one float plane each way
    bpl = BYTES_PER_LU_3D[storage] + (PHI_PLANE_BYTES if remove_fa == 2 else 0.0)
    ach = case.n * bpl / (t / steps) / 1e9
    return dict(mlups=round(mlups, 1), achieved_gbs=round(ach, 1),
                frac=round(ach / HBM_PEAK_GBS, 4), bytes_per_lu=bpl,
                steps=steps, nonfinite=int(d["nonfinite"]), mass_drift_rel=d["mass_drift_rel"],
                ms_per_step=round(1e3 * t / steps, 4), variant=variant,
                kernel=kernel_3d(hip, variant, remove_fa))


def leg_ensemble(torch, W, hip, storage, steps=200, warmup=20):
    """64 droplet cases (64^2..512^2) in one launch per step, against the same
    cases advanced one Simulation at a time."""
    from paper_1110_5004_amd import tune
    cases = W.ensemble(seed=0)
    nodes = sum(c.n for c in cases)
    probe = hip.Simulation(cases, storage=storage)
    rec = tune.tune(probe, steps=20)
    probe.close()
    sim = hip.Simulation(cases, storage=storage)
    sim.set_launch(rec["variant"], rec["grid"], rec["graph_steps"])
    t = time_gpu(torch, sim, steps, warmup)
    bad = sum(int(sim.diagnostics(k)["nonfinite"]) for k in range(len(cases)))
    sim.close()
    out = dict(cases=len(cases), nodes=nodes, batched_mlups=round(nodes * steps / t / 1e6, 1),
               nonfinite=bad)
    if storage == "fp32":
        sims = [hip.Simulation([c], storage=storage) for c in cases]
        for s_ in sims:
            s_.step(warmup)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for s_ in sims:
            s_.step(steps)
        e1.record()
        torch.cuda.synchronize()
        t1 = e0.elapsed_time(e1) / 1e3
        for s_ in sims:
            s_.close()
        out["one_at_a_time_mlups"] = round(nodes * steps / t1 / 1e6, 1)
    return out


def leg_paper(torch, W, hip):
    """The paper's two tests at their own sizes, corrected model, FP32: the
    150x450 falling droplet (20k steps) and the 300x150 splash at Re = 48
    (to t* = 4), each timed over the whole run; the falling droplet also
    reports the spread radius at t = 1.9e4 of both models."""
    from paper_1110_5004_amd import tune
    out = {}
    for name, builder, steps in (("falling150x450", W.paper_falling, 20000),
                                 ("splash300x150_re48", W.paper_splash, 6000)):
        case = builder(remove_fa=1)
        probe = hip.Simulation([case])
        rec = tune.tune(probe, steps=200)
        probe.close()
        sim = hip.Simulation([case])
        sim.set_launch(rec["variant"], rec["grid"], rec["graph_steps"])
        t = time_gpu(torch, sim, steps, 0)
        d = sim.diagnostics()
        sim.close()
        out[name] = dict(steps=steps, seconds=round(t, 4), mlups=round(case.n * steps / t / 1e6, 1),
                         nonfinite=int(d["nonfinite"]))
    radii = {}
    for m in (0, 1):
        sim = hip.Simulation([W.paper_falling(remove_fa=m)])
        sim.step(19000)
        radii[m] = sim.spread_radius()
        sim.close()
    out["falling150x450"]["spread_radius_t19000"] = {"original": round(radii[0], 4),
                                                     "corrected": round(radii[1], 4)}
    return out


# Algorithmic bytes per node of the F_a diagnostic kernels (2-D, FP32 fields):
# phi (or phi and phi^(n-1)), u, and p read once, F_a written: 4 + 4 + 8 + 8.
FA_DIAG_BYTES = 24


def leg_fa_diagnostics(torch, W, hip, reps=20):
    """The two F_a diagnostics (from discrete data, and in Lee and Lin's form)
    on the 4096^2 droplet, FP32, corrected model: each call dumps the fields
    (the same dump lbm_moments_device makes) and runs one node-parallel
    kernel.  The kernel's own time is the call minus the dump alone, priced
    at its algorithmic bytes (FA_DIAG_BYTES per node)."""
    case = W.big_droplet(remove_fa=1)
    sim = hip.Simulation([case])
    sim.step(20)
    prev = sim.moments_device()["phi"].clone()
    sim.step(1)
    n = case.n
    stream = torch.cuda.current_stream()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3 / reps

    t_dump = timed(lambda: sim.moments_device())
    t_ll = timed(lambda: sim.fa_leelin())
    t_fd = timed(lambda: sim.fa_discrete(prev))
    finite = bool(torch.isfinite(sim.fa_leelin()).all()) and \
        bool(torch.isfinite(sim.fa_discrete(prev)).all())
    sim.close()
    out = dict(workload="droplet4096", nodes=n, dump_us=round(t_dump * 1e6, 1), finite=finite)
    for name, t in (("fa_leelin", t_ll), ("fa_discrete", t_fd)):
        k = max(t - t_dump, 1e-9)
        gbs = FA_DIAG_BYTES * n / k / 1e9
        out[name] = dict(call_us=round(t * 1e6, 1), kernel_us=round(k * 1e6, 1),
                         achieved_gbs=round(gbs, 1), frac=round(gbs / HBM_PEAK_GBS, 4))
    return out


def pull_copy_ceiling(torch, hip, lattice, storage, dims, reps=200):
    """Seconds per launch of the pull-copy calibration kernel: the step's
    reads (every population from x - e_i) and writes in the same plane
    layout, without arithmetic.  The practical ceiling of the step's memory
    access pattern on this device."""
    nb = hip.pull_copy_bytes(lattice, storage, dims)
    a = torch.zeros(nb, dtype=torch.uint8, device="cuda")
    b = torch.zeros(nb, dtype=torch.uint8, device="cuda")
    for k in range(10):
        hip.pull_copy_bw(lattice, storage, dims, a if k % 2 == 0 else b, b if k % 2 == 0 else a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for k in range(reps):
        hip.pull_copy_bw(lattice, storage, dims, a if k % 2 == 0 else b, b if k % 2 == 0 else a)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / reps
    del a, b
    return t


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(W, seconds):
    """The FP64 oracle as it stands on the host cores, on the same workload,
    stepping until about `seconds` have passed with all the OpenMP threads it
    gets, then a third as long on one thread."""
    import ctypes
    from oracle import oracle as O
    gomp = ctypes.CDLL("libgomp.so.1")
    case = W.splash_2d(remove_fa=1)
    s = O.Sim(case.params, case.phi0, case.u0, case.p0)
    s.step(1)

    def rate(limit):
        t0 = time.perf_counter()
        steps = 0
        while time.perf_counter() - t0 < limit:
            s.step(2)
            steps += 2
        dt = time.perf_counter() - t0
        return case.n * steps / dt / 1e6, steps, dt

    threads = gomp.omp_get_max_threads()
    value, steps, dt = rate(seconds)
    gomp.omp_set_num_threads(1)
    one, steps1, dt1 = rate(seconds / 3)
    gomp.omp_set_num_threads(threads)
    return dict(value=value, unit="MLUPS", cores=threads, kind="oracle",
                sample=f"{steps} steps of the 1024x512 splash workload (corrected model), "
                       f"{dt:.1f} s, FP64; then {steps1} steps on one thread, {dt1:.1f} s",
                value_one_thread=one, cpu_model=_cpu_model())


STEP_KERNEL_SOURCES = ("lbm_d2q9.hip", "lbm_dev.h", "lbm_lattice.h")


def source_sha():
    """Hash of the sources of the D2Q9 step kernel; traffic figures apply only
    to the kernel they were measured on."""
    import hashlib
    h = hashlib.sha256()
    for name in STEP_KERNEL_SOURCES:
        h.update(name.encode())
        with open(os.path.join(ROOT, "paper_1110_5004_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def traffic_for(kernel_key, seconds_per_launch):
    """Measured HBM-side traffic (rocprofv3 FETCH_SIZE x2 + WRITE_SIZE x1 per
    launch) as GB/s over this run's launch time, or None when the committed
    counters were taken on other kernel sources or another launch shape."""
    try:
        with open(PROFILE_TRAFFIC) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None, None
    e = t.get("entries", {}).get(kernel_key)
    if not e or t.get("source_sha") != source_sha():
        return None, None
    return round(e["bytes_per_launch"] / seconds_per_launch / 1e9, 1), e["bytes_per_launch"]


def main_3d(a, torch, W, hip):
    """The D3Q19 256x256x128 splash alone (profiling of the 3-D path)."""
    r = leg_3d(torch, W, hip, a.storage, a.remove_fa, a.steps, a.warmup, a.variant)
    pc_s = pull_copy_ceiling(torch, hip, hip.D3Q19, a.storage, (256, 256, 128), reps=20)
    step_s = r["ms_per_step"] / 1e3
    print(json.dumps({
        "metric": "lattice updates/s (MLUPS), D3Q19 phase-field step", "value": r["mlups"],
        "unit": "MLUPS", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if a.storage == "fp32" else f"f32 compute, {a.storage} storage",
        "data": "synthetic (seeded 3-D splash initial condition)",
        "config": {"workload": "splash3d", "grid": [256, 256, 128], "lattice": "D3Q19",
                   "bc": "periodic x y, walls z", "storage": a.storage,
                   "remove_fa": a.remove_fa},
        "roofline": {"bound": "hbm", "achieved": r["achieved_gbs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": r["frac"], "traffic": None,
                     "bytes_per_lu": r["bytes_per_lu"],
                     "kernel": r["kernel"], "variant": r["variant"],
                     "pull_copy_us": round(pc_s * 1e6, 2),
                     "frac_of_pull_copy": round(pc_s / step_s, 4)},
        "check": {"mass_drift_rel": r["mass_drift_rel"], "nonfinite": r["nonfinite"]},
    }), flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "one GPU only: the step has no multi-GPU path, --gpus must be 1"}))
        sys.exit(2)
    import torch
    import paper_1110_5004_amd as hip
    import workloads as W
    hip.lib()
    if a.workload == "splash3d":
        main_3d(a, torch, W, hip)
        return
    if a.workload == "fa_diagnostics":
        print(json.dumps({"fa_diagnostics": leg_fa_diagnostics(torch, W, hip)}), flush=True)
        return

    main_leg = leg(torch, W, hip, a.storage, a.remove_fa, a.steps, a.warmup, a.workload,
                   a.variant)
    bpl = BYTES_PER_LU[a.storage] + (PHI_PLANE_BYTES if a.remove_fa == 2 else 0.0)
    achieved = main_leg["nodes"] * bpl / (main_leg["seconds"] / a.steps) / 1e9
    key = f"{a.workload}_{a.storage}_rf{a.remove_fa}_v{main_leg['variant']}"
    step_s = main_leg["seconds"] / a.steps
    traffic, traffic_bytes = traffic_for(key, step_s)
    dims = (1024, 512) if a.workload == "splash1024x512" else (4096, 4096)
    pc_s = pull_copy_ceiling(torch, hip, hip.D2Q9, a.storage, dims)
    out = {
        "metric": "lattice updates/s (MLUPS), fused D2Q9 phase-field step",
        "value": round(main_leg["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(main_leg["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if a.storage == "fp32" else f"f32 compute, {a.storage} storage",
        "data": "synthetic (seeded splash initial condition)",
        "config": ({"workload": "splash1024x512", "grid": [1024, 512], "lattice": "D2Q9",
                    "bc": "periodic x, walls y", "storage": a.storage,
                    "remove_fa": a.remove_fa, "steps_in_job": 20000}
                   if a.workload == "splash1024x512" else
                   {"workload": "droplet4096", "grid": [4096, 4096], "lattice": "D2Q9",
                    "bc": "periodic", "storage": a.storage, "remove_fa": a.remove_fa}),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "traffic_bytes_per_launch": traffic_bytes,
                     "bytes_per_lu": bpl, "kernel": "k_tile (fused D2Q9 step)",
                     "variant": main_leg["variant"],
                     # the same reads and writes without arithmetic (lbm_pull_copy_bw)
                     "pull_copy_us": round(pc_s * 1e6, 2),
                     "frac_of_pull_copy": round(pc_s / step_s, 4)},
        "check": {"mass_drift_rel": main_leg["mass_drift_rel"],
                  "nonfinite": main_leg["nonfinite"], "umax": main_leg["umax"]},
    }
    if not a.no_extra:
        extra = {}
        other = [0, 1, 2]
        other.remove(a.remove_fa)
        for st, rf in [("fp16", a.remove_fa), ("bf16", a.remove_fa)] + \
                [(a.storage, r) for r in other]:
            r = leg(torch, W, hip, st, rf, a.steps, a.warmup, a.workload)
            bpl_rf = BYTES_PER_LU[st] + (PHI_PLANE_BYTES if rf == 2 else 0.0)
            ach = r["nodes"] * bpl_rf / (r["seconds"] / a.steps) / 1e9
            extra[f"{st}_rf{rf}"] = dict(mlups=round(r["mlups"], 1),
                                         achieved_gbs=round(ach, 1),
                                         frac=round(ach / HBM_PEAK_GBS, 4),
                                         nonfinite=r["nonfinite"],
                                         mass_drift_rel=r["mass_drift_rel"])
        out["variants"] = extra
        out["d3q19_splash256x256x128"] = {f"{st}_rf{rf}": leg_3d(torch, W, hip, st, rf)
                                          for st, rf in (("fp16", 1), ("fp16", 0), ("fp32", 1),
                                                         ("fp32", 0), ("fp32", 2))}
        out["ensemble64"] = {st: leg_ensemble(torch, W, hip, st) for st in ("fp32", "fp16")}
        out["paper_experiments"] = leg_paper(torch, W, hip)
        out["fa_diagnostics"] = leg_fa_diagnostics(torch, W, hip)
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(W, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
