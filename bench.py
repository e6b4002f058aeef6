"""Benchmark of the phase-field LBM step on one MI355X.

Headline workload: droplet splash on a thin film in 3-D, 256 x 256 x 128
D3Q19 (periodic x and y, bounce-back walls in z), FP32 arithmetic with the
populations stored in FP16, corrected model (the whole path including the
lap mu stencil of the -F_a correction).  A step is one lattice time step of
the whole grid.  Inputs are resident in HBM before timing starts, and the
step graph is captured before the timed window.

Prints one JSON line: MLUPS (lattice updates per second / 1e6) of the
headline, the roofline of its step kernel (algorithmic bytes per lattice
update: every stored population read once and written once, 156 B with
16-bit storage (18 f and 19 g at 2 B, f_0 at 4 B) and 304 B with FP32
storage), the FP64 CPU oracle timed on a bounded sample of the same
workload, and the other legs: both switch positions, FP32 and BF16 storage,
the correction from data, the 2-D workloads, the 64-case ensemble, the
paper's own experiments and the two F_a diagnostics.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "lattice updates/s (MLUPS) & % of HBM peak; FP16-storage vs FP32 at equal error"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per lattice update (each population read once and written
# once); FP32 prices the populations alone (the 2-byte low part of f_0 that
# the FP32 layout adds is not counted)
BYTES_PER_LU = {2: {"fp32": 144.0, "fp16": 76.0, "bf16": 76.0},
                3: {"fp32": 304.0, "fp16": 156.0, "bf16": 156.0}}
# the correction from data also reads and writes one float of phi per node
PHI_PLANE_BYTES = 8.0
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "traffic.json")
WORKLOADS = ("splash3d", "splash1024x512", "droplet4096", "fa_diagnostics")
# sources of the step kernels of each lattice: committed counters apply only
# to the kernel they were taken on
KERNEL_SOURCES = {2: ("lbm_d2q9.hip", "lbm_dev.h", "lbm_lattice.h"),
                  3: ("lbm_d3q19.hip", "lbm_d3q19_march.hip", "lbm_d3q19_lean.h",
                      "lbm_d3q19_addr.h", "lbm_dev.h", "lbm_lattice.h")}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--storage", default="fp16", choices=["fp32", "fp16", "bf16"])
    ap.add_argument("--remove-fa", type=int, default=1, choices=[0, 1, 2])
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="skip the other legs")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--workload", default="splash3d", choices=WORKLOADS,
                    help="splash3d (the benchmark: 256x256x128 D3Q19 splash), "
                         "splash1024x512 (the 2-D splash), droplet4096 (4096^2 2-D "
                         "droplet, HBM-bound) or fa_diagnostics (the two F_a "
                         "diagnostics alone)")
    ap.add_argument("--variant", type=int, default=-1,
                    help="tile variant; -1 = autotuned")
    return ap.parse_args()


def make_case(W, workload, remove_fa):
    if workload == "splash3d":
        return W.splash_3d(remove_fa=remove_fa)
    if workload == "droplet4096":
        return W.big_droplet(remove_fa=remove_fa)
    return W.splash_2d(remove_fa=remove_fa)


def time_steps(torch, sim, steps, warmup):
    """Seconds of `steps` steps after `warmup` untimed ones.  The step graph
    is captured first (lbm_prepare), so the timed window holds graph replays
    and eager launches only; HIP events on the stream the library launches
    on (the current stream at Simulation creation)."""
    sim.prepare()
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


def tuned_sim(hip, cases, storage, variant=-1, tune_steps=32):
    """A Simulation of `cases` with the launch shape of `variant`, or the one
    the autotuner picks on a scratch copy (so the timed run starts from the
    initial state)."""
    from paper_1110_5004_amd import tune
    if variant >= 0:
        rec = dict(variant=variant, grid=0, graph_steps=16)
    else:
        probe = hip.Simulation(cases, storage=storage)
        rec = tune.tune(probe, steps=tune_steps)
        probe.close()
    sim = hip.Simulation(cases, storage=storage)
    sim.set_launch(rec["variant"], rec["grid"], rec["graph_steps"])
    return sim


def source_sha(dim):
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[dim]:
        h.update(name.encode())
        with open(os.path.join(ROOT, "paper_1110_5004_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def traffic_for(key, dim, seconds_per_launch):
    """Measured HBM-side traffic of the step kernel (rocprofv3 FETCH_SIZE x2 +
    WRITE_SIZE x1 per launch, committed under profiles/) as GB/s over this
    run's launch time, or (None, None) when the counters were taken on other
    kernel sources or another launch shape."""
    try:
        with open(PROFILE_TRAFFIC) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None, None
    e = t.get("entries", {}).get(key)
    if not e or e.get("source_sha") != source_sha(dim):
        return None, None
    return round(e["bytes_per_launch"] / seconds_per_launch / 1e9, 1), e["bytes_per_launch"]


def kernel_name(hip, dim, variant, params, storage):
    """The step kernel a launch variant runs, chosen as the launcher chooses:
    the D3Q19 fused step drops the lap mu stage when the Eq. 5 coefficient
    (d rho / d phi theta_M, kept only by remove_fa = 1) is zero."""
    if dim == 2:
        return "k_tile (fused D2Q9 step)"
    form = hip.variants(hip.D3Q19)[variant][4]
    rf = params["remove_fa"]
    if form == hip.FORM_TWO and storage != "fp32":
        return ("k3_pull + k3_fcm (two-kernel D3Q19 step, 16-bit storage"
                + (", correction from data)" if rf == 2 else ")"))
    if form != hip.FORM_FUSED:
        return "k3_pull + k3_fields_t + k3_collide"
    coef_zero = rf != 1 or params["theta_m"] == 0.0 or params["rho_l"] == params["rho_g"]
    if storage != "fp32":
        if rf == 2:
            return "k3_pull + k3_fields_t + k3_collide (correction from data, 16-bit)"
        return ("k3_march (fused D3Q19 step, 16-bit storage"
                + (", no lap mu stage)" if coef_zero else ")"))
    if rf == 2:
        return "k3_slab (fused D3Q19 step, correction from data)"
    if coef_zero:
        return "k3_slab2 (fused D3Q19 step without the Eq. 5 term)"
    return "k3_slab (fused D3Q19 step)"


def leg(torch, W, hip, workload, storage, remove_fa, steps, warmup, variant=-1):
    """One timed run of a workload; MLUPS, step time and the roofline
    fraction at the algorithmic bytes."""
    case = make_case(W, workload, remove_fa)
    dim = 3 if workload == "splash3d" else 2
    sim = tuned_sim(hip, [case], storage, variant, tune_steps=32 if case.n > 4e6 else 160)
    t = time_steps(torch, sim, steps, warmup)
    d = sim.diagnostics()
    variant = sim.get_launch()[0]
    sim.close()
    bpl = BYTES_PER_LU[dim][storage] + (PHI_PLANE_BYTES if remove_fa == 2 else 0.0)
    step_s = t / steps
    ach = case.n * bpl / step_s / 1e9
    return dict(mlups=round(case.n * steps / t / 1e6, 1), ms_per_step=round(1e3 * step_s, 5),
                achieved_gbs=round(ach, 1), frac=round(ach / HBM_PEAK_GBS, 4),
                bytes_per_lu=bpl, nodes=case.n, variant=variant,
                kernel=kernel_name(hip, dim, variant, case.params, storage),
                mass_drift_rel=d["mass_drift_rel"], nonfinite=int(d["nonfinite"]),
                umax=d["umax"])


def leg_ensemble(torch, W, hip, storage, steps=200, warmup=20):
    """64 droplet cases (64^2..512^2) in one launch per step, against the same
    cases advanced one Simulation at a time."""
    cases = W.ensemble(seed=0)
    nodes = sum(c.n for c in cases)
    sim = tuned_sim(hip, cases, storage, tune_steps=32)
    t = time_steps(torch, sim, steps, warmup)
    bad = sum(int(sim.diagnostics(k)["nonfinite"]) for k in range(len(cases)))
    sim.close()
    ach = nodes * BYTES_PER_LU[2][storage] / (t / steps) / 1e9
    out = dict(cases=len(cases), nodes=nodes, batched_mlups=round(nodes * steps / t / 1e6, 1),
               achieved_gbs=round(ach, 1), frac=round(ach / HBM_PEAK_GBS, 4), nonfinite=bad)
    if storage == "fp32":
        sims = [hip.Simulation([c], storage=storage) for c in cases]
        for s_ in sims:
            s_.prepare()
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
    out = {}
    for name, builder, steps in (("falling150x450", W.paper_falling, 20000),
                                 ("splash300x150_re48", W.paper_splash, 6000)):
        case = builder(remove_fa=1)
        sim = tuned_sim(hip, [case], "fp32", tune_steps=160)
        t = time_steps(torch, sim, steps, 0)
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


def pull_copy_ceiling(torch, hip, lattice, storage, dims, reps=50):
    """Seconds per launch of the pull-copy calibration kernel: the step's
    reads (every population from x - e_i) and writes in the same plane
    layout, without arithmetic.  The practical ceiling of the step's memory
    access pattern on this device."""
    nb = hip.pull_copy_bytes(lattice, storage, dims)
    a = torch.zeros(nb, dtype=torch.uint8, device="cuda")
    b = torch.zeros(nb, dtype=torch.uint8, device="cuda")
    for k in range(6):
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


def copy_ceiling_gbs(torch, hip, nbytes=1 << 31, reps=20):
    """GB/s (read + written) of lbm_copy_bw on two HBM-resident buffers of
    nbytes: the plain-copy ceiling of the device (16-byte non-temporal loads
    and stores, four per thread and round)."""
    n = nbytes // 4
    a = torch.zeros(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        hip.copy_bw(a, b)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        hip.copy_bw(a, b)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / reps
    del a, b
    return 2.0 * nbytes / t / 1e9


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(W, workload, remove_fa, seconds):
    """The FP64 oracle as it stands on the host cores, on the same workload:
    steps until about `seconds` have passed, with all the OpenMP threads it
    gets (the creation of its state is not timed)."""
    import ctypes
    from oracle import oracle as O
    gomp = ctypes.CDLL("libgomp.so.1")
    case = make_case(W, workload, remove_fa)
    s = O.Sim(case.params, case.phi0, case.u0, case.p0)
    threads = gomp.omp_get_max_threads()
    t0 = time.perf_counter()
    steps = 0
    while time.perf_counter() - t0 < seconds:
        s.step(1)
        steps += 1
    dt = time.perf_counter() - t0
    del s
    return dict(value=round(case.n * steps / dt / 1e6, 3), unit="MLUPS", cores=threads,
                kind="oracle",
                sample=f"{steps} steps of the {case.name} workload (remove_fa={remove_fa}), "
                       f"{dt:.1f} s, FP64, {threads} OpenMP threads",
                cpu_model=_cpu_model())


def config_of(workload, storage, remove_fa):
    if workload == "splash3d":
        return {"workload": "splash3d256x256x128", "grid": [256, 256, 128], "lattice": "D3Q19",
                "bc": "periodic x y, walls z", "storage": storage, "remove_fa": remove_fa,
                "steps_in_job": 5000}
    if workload == "droplet4096":
        return {"workload": "droplet4096", "grid": [4096, 4096], "lattice": "D2Q9",
                "bc": "periodic", "storage": storage, "remove_fa": remove_fa}
    return {"workload": "splash1024x512", "grid": [1024, 512], "lattice": "D2Q9",
            "bc": "periodic x, walls y", "storage": storage, "remove_fa": remove_fa,
            "steps_in_job": 20000}


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "one GPU only: the step has no multi-GPU path, --gpus must be 1"}))
        sys.exit(2)
    import torch
    import paper_1110_5004_amd as hip
    import workloads as W
    hip.lib()
    if a.workload == "fa_diagnostics":
        print(json.dumps({"fa_diagnostics": leg_fa_diagnostics(torch, W, hip)}), flush=True)
        return

    dim = 3 if a.workload == "splash3d" else 2
    main_leg = leg(torch, W, hip, a.workload, a.storage, a.remove_fa, a.steps, a.warmup,
                   a.variant)
    step_s = main_leg["ms_per_step"] / 1e3
    key = f"{a.workload}_{a.storage}_rf{a.remove_fa}_v{main_leg['variant']}"
    traffic, traffic_bytes = traffic_for(key, dim, step_s)
    dims = {"splash3d": (256, 256, 128), "droplet4096": (4096, 4096, 1),
            "splash1024x512": (1024, 512, 1)}[a.workload]
    lattice = hip.D3Q19 if dim == 3 else hip.D2Q9
    pc_s = pull_copy_ceiling(torch, hip, lattice, a.storage, dims[:dim])
    copy_gbs = copy_ceiling_gbs(torch, hip)
    out = {
        "metric": METRIC,
        "value": main_leg["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": main_leg["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if a.storage == "fp32" else f"f32 compute, {a.storage} storage",
        "data": "synthetic (seeded splash initial condition)" if a.workload != "droplet4096"
                else "synthetic (seeded droplet initial condition)",
        "config": config_of(a.workload, a.storage, a.remove_fa),
        "roofline": {"bound": "hbm", "achieved": main_leg["achieved_gbs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": main_leg["frac"], "traffic": traffic,
                     "traffic_bytes_per_launch": traffic_bytes,
                     "bytes_per_lu": main_leg["bytes_per_lu"], "kernel": main_leg["kernel"],
                     "variant": main_leg["variant"],
                     # the same reads and writes without arithmetic (lbm_pull_copy_bw)
                     "pull_copy_us": round(pc_s * 1e6, 2),
                     "frac_of_pull_copy": round(pc_s / step_s, 4),
                     # a plain 2 GiB copy (lbm_copy_bw): the device's HBM copy ceiling
                     "copy_gbs": round(copy_gbs, 1),
                     "frac_of_copy": round(main_leg["achieved_gbs"] / copy_gbs, 4)},
        "check": {"mass_drift_rel": main_leg["mass_drift_rel"],
                  "nonfinite": main_leg["nonfinite"], "umax": main_leg["umax"]},
    }
    if not a.no_extra:
        legs = {}
        if a.workload == "splash3d":
            for st, rf in (("fp16", 0), ("fp32", 1), ("fp32", 0), ("bf16", 1), ("fp32", 2),
                           ("fp16", 2)):
                if (st, rf) != (a.storage, a.remove_fa):
                    legs[f"splash3d_{st}_rf{rf}"] = leg(torch, W, hip, "splash3d", st, rf,
                                                        100, 10)
        for wl, steps in (("splash1024x512", 2000), ("droplet4096", 100)):
            for st in ("fp32", "fp16"):
                legs[f"{wl}_{st}_rf1"] = leg(torch, W, hip, wl, st, 1, steps, 20)
        out["legs"] = legs
        # FP16 against FP32 storage on the headline workload (error bounds: tests)
        l32 = legs.get(f"splash3d_fp32_rf{a.remove_fa}")
        if a.workload == "splash3d" and l32 and a.storage == "fp16":
            out["fp16_over_fp32_mlups"] = round(main_leg["mlups"] / l32["mlups"], 3)
        out["ensemble64"] = {st: leg_ensemble(torch, W, hip, st) for st in ("fp32", "fp16")}
        out["paper_experiments"] = leg_paper(torch, W, hip)
        out["fa_diagnostics"] = leg_fa_diagnostics(torch, W, hip)
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(W, a.workload, a.remove_fa, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
