"""FIRE 2.0 hot-path benchmark on one MI355X.

A step is one full FIRE 2.0 relaxation of the workload to fmax < 1e-6 (all
hot-path stages: stage-in and cell sort, neighbour list, force passes with
fused reductions, FIRE control and update), starting from the same
HBM-resident positions each time.

Default workload (the headline configuration): LJ, FCC 32x32x32 cells
(131,072 sites, 655 vacancies -> 130,417 atoms), Gaussian noise 0.05 sigma,
FP64 path; the mixed-precision path is run on the same input beside it.

Prints ONE JSON line.  value = atom-force-evals/s = atoms * force evaluations
/ wall time of the K timed relaxations.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "atom-force-evals/s + FIRE2 steps/s to fmax 1e-6; mixed/batched vs FP64 plain"
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3

# Algorithmic cost of one force evaluation per atom (each in-range pair counted
# once, FCC neighbour shells): LJ rc = 2.5 sigma -> 54 neighbours = 27 pairs of
# ~25 flop (separation 3, r^2 5, 1/r^2 1, r^-6 3, force factor 4, F_i and F_j
# updates 6, plus the cutoff test); Gupta r_out = 5 A -> 42 neighbours = 21
# pairs of ~125 flop (FP64, two exponentials and a square root).  Bytes: positions read once, velocities
# read for P = F.v, forces written (3 x 8 B each); the EAM form adds F'(rho)
# written and read (2 x 8 B).  Stillinger-Weber on diamond Si: 4 neighbours
# -> 2 pairs of ~70 flop (two exponentials, a power) and 6 triplets of ~90 flop
# (cosine, both end gradients, the radial factors), each term counted once;
# bytes as for LJ (the short lists are the implementation's, not the method's).
ALG = {
    "lj": {"bytes": 72.0, "flops": 27.0 * 25.0, "kernel": "k_lj_force", "tag": "k_lj_force_global"},
    "gupta": {"bytes": 120.0, "flops": 21.0 * 165.0, "kernel": "k_gupta_density + k_gupta_force",
              "tag": "k_gupta_global"},
    "sw": {"bytes": 72.0, "flops": 2.0 * 70.0 + 6.0 * 90.0, "kernel": "k_sw_short + k_sw_force",
           "tag": "k_sw_global"},
}
# The LDS-staged loop folds the update into the first pass of each iteration
# (the kernel that dominates a relaxation): per atom it also reads the
# position at the last list build and writes the new position and velocity
# (x, v, F read; x, v, F written; x_ref read: 7 x 24 B), and does ~20 more flop.
FUSED = {
    "lj": {"bytes": 168.0, "flops": 27.0 * 25.0 + 20.0, "kernel": "k_lj_force<double, true, false, true>",
           "tag": "k_lj_force_fused"},
    "gupta": {"bytes": 216.0, "flops": 21.0 * 165.0 + 20.0,
              "kernel": "k_gupta_density<double, true, true> + k_gupta_force<double, true, false>",
              "tag": "k_gupta_fused"},
}


FP32_KERNEL = {
    "lj": "k_lj_force<float, true, false, true>",
    "gupta": "k_gupta_density<float, true, true> + k_gupta_force<float, true, false>",
}


def with_tile(kernel: str, tuning: str) -> str:
    """The EAM-form kernels carry their tile size (256 or 512 atoms, the
    tuner's choice) as a last template argument."""
    if "k_gupta" not in kernel:
        return kernel
    tile = 512 if "512-atom tiles" in (tuning or "") else 256
    return kernel.replace(", true>", f", true, {tile}>").replace(", false>", f", false, {tile}>")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash() -> str:
    h = hashlib.sha1()
    for f in ("fire2.hip", "fire2_internal.h"):
        with open(os.path.join(ROOT, "paper_1908_02038_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:12]


def load_traffic(tag: str, workload: str):
    """HBM traffic per launch from a committed rocprofv3 counter summary, or
    None when the kernel source changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{tag}_{workload}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_hash") != source_hash():
        return None
    return rec.get("bytes_per_launch")


def load_limiter(tag: str, workload: str):
    """What the hardware counters say binds the dominant kernel (VALU busy
    share, share of wave life spent waiting, resident waves per SIMD), from a
    committed rocprofv3 counter summary, or None when the kernel source
    changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"counters_{tag}_{workload}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_hash") != source_hash():
        return None
    return {k: rec[k] for k in ("valu_busy", "wait_share", "lds_wait_share", "waves_per_simd", "reading")}


def make_system(name: str):
    from paper_1908_02038_amd import inputs
    return inputs.WORKLOADS[name]()


def time_relaxations(ctx, pos0_dev, s, steps: int, warmup: int, max_steps: int):
    import torch
    work = torch.empty_like(pos0_dev)
    res = None
    for _ in range(warmup):
        work.copy_(pos0_dev)
        res = ctx.fire_minimize_dev(work, s.box, s.potential, s.tol, max_steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for _ in range(steps):
        work.copy_(pos0_dev)
        results.append(ctx.fire_minimize_dev(work, s.box, s.potential, s.tol, max_steps))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dt, results, work


def kernel_time_ms(ctx, reps: int) -> float:
    """Average duration of one force evaluation (the dominant kernel), HIP
    events on the stream the kernels are launched on."""
    import torch
    stream = torch.cuda.current_stream()
    ctx.fire_repeat_forces_dev(3)  # warm
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    ctx.fire_repeat_forces_dev(reps)
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def bench_batched(args):
    """The batched form: 512 independent EAM-form relaxations (500-4000 atoms,
    clusters and periodic boxes) in one persistent launch, positions resident
    in HBM, against the plain FP64 single-system path on a sample of the same
    systems, one relaxation after another."""
    import torch
    from paper_1908_02038_amd import api, inputs
    systems = inputs.batched()
    pot, fire, tol = systems[0].potential, systems[0].fire, systems[0].tol
    offs = np.cumsum([0] + [len(s.pos) for s in systems])
    boxes = [s.box for s in systems]
    src = torch.tensor(np.concatenate([s.pos for s in systems]), dtype=torch.float64, device="cuda")
    work = torch.empty_like(src)
    ctx = api.Context(0, fire)
    for _ in range(max(1, args.warmup)):  # the first call also autotunes the team shape
        work.copy_(src)
        ctx.fire_minimize_batched_dev(work, offs, boxes, pot, tol, args.max_steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = None
    for _ in range(args.steps):
        work.copy_(src)
        res = ctx.fire_minimize_batched_dev(work, offs, boxes, pot, tol, args.max_steps)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    tuning = ctx.fire_tuning_info()
    ctx.close()
    # the same batch with FP32 pair terms until each system's criterion falls
    # below its switch, then FP64
    ctxm = api.Context(0, fire, precision="mixed")
    for _ in range(max(1, args.warmup)):
        work.copy_(src)
        ctxm.fire_minimize_batched_dev(work, offs, boxes, pot, tol, args.max_steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        work.copy_(src)
        res_m = ctxm.fire_minimize_batched_dev(work, offs, boxes, pot, tol, args.max_steps)
    torch.cuda.synchronize()
    dtm = (time.perf_counter() - t0) / args.steps
    ctxm.close()
    atom_evals = sum(len(s.pos) * r["force_evals"] for s, r in zip(systems, res))
    iters = sum(r["iterations"] for r in res)
    stops = [r["stop"] for r in res]
    # plain FP64 path, one system after another, on every 16th system
    sample = list(range(0, len(systems), 16))
    ctx = api.Context(0, fire, precision="fp64")
    dev = [torch.tensor(systems[k].pos, dtype=torch.float64, device="cuda") for k in sample]
    w = [torch.empty_like(d) for d in dev]
    for d, x in zip(dev, w):
        x.copy_(d)
    ctx.fire_minimize_dev(w[0], systems[sample[0]].box, pot, tol, args.max_steps)  # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain_evals = plain_iters = 0
    for k, d, x in zip(sample, dev, w):
        x.copy_(d)
        r = ctx.fire_minimize_dev(x, systems[k].box, pot, tol, args.max_steps)
        plain_evals += len(systems[k].pos) * r["force_evals"]
        plain_iters += r["iterations"]
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    ctx.close()
    val = atom_evals / dt
    plain = plain_evals / tp
    log(f"[bench] batched: {len(systems)} systems, {offs[-1]} atoms, {dt * 1e3:.1f} ms per batch, "
        f"{val:.3e} atom-force-evals/s; plain FP64 path on {len(sample)} of them: {plain:.3e}")
    return {
        "workload": f"{len(systems)} Gupta systems, {int(offs[-1])} atoms, 500-4000 atoms each",
        "value": val,
        "unit": "atom-force-evals/s",
        "ms_per_batch": dt * 1e3,
        "steps_per_s": iters / dt,
        "all_converged": all(x == "converged" for x in stops),
        "max_iterations": max(r["iterations"] for r in res),
        "plain_fp64_value": plain,
        "plain_fp64_steps_per_s": plain_iters / tp,
        "plain_sample": f"every 16th system ({len(sample)}), relaxed one after another by fire_minimize_dev",
        "speedup_vs_plain": val / plain,
        "tuning": tuning,
        "mixed": {"ms_per_batch": dtm * 1e3,
                  "value": sum(len(s.pos) * r["force_evals"] for s, r in zip(systems, res_m)) / dtm,
                  "all_converged": all(r["stop"] == "converged" for r in res_m),
                  "max_iterations": max(r["iterations"] for r in res_m)},
    }


def measure_config(name: str, precision: str, steps: int, warmup: int, max_steps: int, kernel_reps: int = 20):
    """One workload at one precision: timed relaxations (inputs resident in
    HBM), iterations, and the force evaluation's HIP-event time against the
    algorithmic bytes and flops of the pass that dominates the loop."""
    import torch
    from paper_1908_02038_amd import api
    s = make_system(name)
    n = len(s.pos)
    kind = s.potential["kind"]
    pos0 = torch.tensor(s.pos, dtype=torch.float64, device="cuda")
    ctx = api.Context(0, s.fire, precision=precision)
    dt, res, _ = time_relaxations(ctx, pos0, s, steps, warmup, max_steps)
    kt = kernel_time_ms(ctx, kernel_reps)
    tuning = ctx.fire_tuning_info()
    ctx.close()
    r = res[-1]
    staged = os.environ.get("FIRE_LDS", "1") != "0" and kind != "sw"
    alg = FUSED[kind] if staged else ALG[kind]
    hbm = alg["bytes"] * n / (kt * 1e-3) / 1e9
    alu = alg["flops"] * n / (kt * 1e-3) / 1e12
    peak_alu = PEAK_FP64_TFLOPS if precision == "fp64" else PEAK_FP32_TFLOPS
    return {
        "atoms": n, "potential": kind, "precision": precision, "fmax_tol": s.tol,
        "value": n * sum(x["force_evals"] for x in res) / dt, "unit": "atom-force-evals/s",
        "ms_per_relaxation": dt / steps * 1e3, "steps_per_s": sum(x["iterations"] for x in res) / dt,
        "iterations": r["iterations"], "iterations_fp32": r["iterations_low"], "rebuilds": r["rebuilds"],
        "stop": r["stop"], "energy_per_atom": r["energy_per_atom"], "fmax": r["fmax"],
        "force_pass_us": kt * 1e3,
        "force_pass_kernel": with_tile(alg["kernel"] if precision == "fp64" or kind == "sw" else FP32_KERNEL[kind],
                                       tuning),
        "force_pass_hbm_frac_alg": hbm / PEAK_HBM_GBS, "force_pass_hbm_GBs_alg": hbm,
        "force_pass_alu_frac_alg": alu / peak_alu, "force_pass_TFLOPs_alg": alu,
        "note": "force pass timed at the relaxed positions with the run's first pair precision"
                if precision != "fp64" else "",
        "tuning": tuning,
    }


def other_configs(args):
    """The other single-system configurations, one line each (the headline's
    LJ bulk is the top-level record): the 255-atom LJ crystal to 1e-8, the
    253,440-atom EAM-form bulk in FP64 and mixed, the 2,037,760-atom EAM-form
    slab in mixed precision (its passes have enough atoms per CU to press on
    HBM), and the 32,763-atom Stillinger-Weber Si slab."""
    out = {}
    plan = [("lj_small", "fp64", 3, 1), ("gupta_bulk", "fp64", 3, 1), ("gupta_bulk", "mixed", 3, 1),
            ("gupta_slab", "mixed", 1, 1), ("si_slab", "fp64", 3, 1)]
    for name, prec, steps, warm in plan:
        r = measure_config(name, prec, steps, warm, args.max_steps)
        out[f"{name}_{prec}"] = r
        log(f"[bench] {name} {prec}: {r['ms_per_relaxation']:.1f} ms/relaxation, {r['iterations']} iterations, "
            f"stop {r['stop']}, force pass {r['force_pass_us']:.1f} us ({r['force_pass_hbm_frac_alg']:.3f} of HBM alg, "
            f"{r['force_pass_alu_frac_alg']:.3f} of {prec} VALU alg)")
    return out


COPY_BYTES = 256 << 20


def kernel_only(args, s, pos0):
    """Force pass alone (lists built from the workload's start positions as a
    relaxation builds them; FIRE_LIST_CLASSES fixes the list order without
    the tuner's timing runs), then one plain device copy of COPY_BYTES: the
    copy reads and writes exactly COPY_BYTES each, which calibrates the byte
    counters of the same run."""
    import torch
    from paper_1908_02038_amd import api
    ctx = api.Context(0, s.fire, precision=args.kernel_precision)
    # a minimisation of no steps: lists built (and the list order chosen) as
    # a relaxation of this workload starts
    work = pos0.clone()
    ctx.fire_minimize_dev(work, s.box, s.potential, s.tol, 0)
    torch.cuda.synchronize()
    kt = kernel_time_ms(ctx, args.kernel_reps)
    ctx.close()
    a = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"kernel_only": args.workload, "precision": args.kernel_precision, "atoms": len(s.pos),
                      "ms_per_launch": kt,
                      "reps": args.kernel_reps, "copy_bytes": COPY_BYTES}), flush=True)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(s, budget_s: float):
    """The oracle as it stands (pairs found through its cell grid, O(N) per
    evaluation; OpenMP over atoms) on a bounded sample: the first FIRE 2.0
    iterations of the same workload, on all of the host's threads and on one.
    Its results do not depend on the thread count."""
    import oracle
    n = len(s.pos)
    out = {"unit": "atom-force-evals/s", "kind": "oracle", "cpu_model": cpu_model(), "nproc": os.cpu_count()}
    all_threads = oracle.threads()
    legs = {}
    with oracle.cells():
        for label, threads, share in (("all_cores", all_threads, 0.6), ("one_core", 1, 0.4)):
            oracle.set_threads(threads)
            t0 = time.perf_counter()
            oracle.energy_forces(s.pos, s.box, s.potential)
            t1 = time.perf_counter() - t0
            steps = max(1, min(500, int(share * budget_s / max(t1, 1e-9)) - 1))
            t0 = time.perf_counter()
            r = oracle.fire_minimize(s.pos, s.box, s.potential, s.fire, s.tol, steps)
            dt = time.perf_counter() - t0
            legs[label] = {"threads": threads, "iterations": r["iterations"], "force_evals": r["force_evals"],
                           "seconds": dt, "value": n * r["force_evals"] / dt, "steps_per_s": r["iterations"] / dt}
    oracle.set_threads(all_threads)
    a = legs["all_cores"]
    out.update({
        "value": a["value"],
        "cores": a["threads"],
        "steps_per_s": a["steps_per_s"],
        "one_core": legs["one_core"],
        "all_cores": a,
        "sample": f"the first {a['iterations']} FIRE 2.0 iterations ({a['force_evals']} force evaluations) of the full "
                  f"{n}-atom workload on {a['threads']} threads ({a['seconds']:.1f} s), and "
                  f"{legs['one_core']['iterations']} on one thread ({legs['one_core']['seconds']:.1f} s); "
                  f"pairs through the oracle's cell grid",
    })
    return out


def relax_once(ctx, pos0_dev, s, max_steps: int, fire: dict):
    """One relaxation of system s with FIRE parameters `fire` (after one
    untimed run with the same parameters): the result and its wall time."""
    import torch
    ctx.fire_set_params(fire)
    work = torch.empty_like(pos0_dev)
    work.copy_(pos0_dev)
    ctx.fire_minimize_dev(work, s.box, s.potential, s.tol, max_steps)
    work.copy_(pos0_dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = ctx.fire_minimize_dev(work, s.box, s.potential, s.tol, max_steps)
    torch.cuda.synchronize()
    return r, time.perf_counter() - t0


def study_integrators(args):
    """Force evaluations to the workload's tolerance with FIRE 2.0 under each
    integrator of Sec. 3.1 (Algorithms 3, 4 and 6) and with the original FIRE
    (Algorithm 1): the paper's integrator comparison and its FIRE / FIRE 2.0
    ratios, on the synthetic workloads."""
    import torch
    from paper_1908_02038_amd import api
    rows = []
    for name in ("lj_bulk", "gupta_bulk", "si_slab"):
        s = make_system(name)
        pos0 = torch.tensor(s.pos, dtype=torch.float64, device="cuda")
        ctx = api.Context(0, s.fire, precision="fp64")
        for variant, integrator in (("fire2", "eulerimplicit"), ("fire2", "eulerexplicit"), ("fire2", "verlet"),
                                    ("fire1", "eulerimplicit"), ("fire1", "eulerexplicit")):
            r, dt = relax_once(ctx, pos0, s, args.max_steps, dict(s.fire, variant=variant, integrator=integrator))
            rows.append({"workload": name, "variant": variant, "integrator": integrator, "stop": r["stop"],
                         "iterations": r["iterations"], "force_evals": r["force_evals"], "fmax": r["fmax"],
                         "energy_per_atom": r["energy_per_atom"], "ms": dt * 1e3})
            log(f"[study] {name} {variant} {integrator}: {r['stop']} after {r['force_evals']} evaluations, "
                f"{dt * 1e3:.1f} ms, E/N {r['energy_per_atom']:.12f}")
        ctx.close()
    return {"study": "integrators", "max_steps": args.max_steps, "rows": rows}


def study_sweep(args):
    """FIRE 2.0 parameter study of Sec. 5.4 (Fig. 3) on the Si slab (the stand-in for the
    paper's Si vacancy case): force evaluations to the tolerance as a function
    of alpha0 for several tmax at dt = 1 fs, and of tmax for several dt at
    alpha0 = 0.15.  Runs that stop without converging report their stop."""
    import torch
    from paper_1908_02038_amd import api
    s = make_system("si_slab")
    pos0 = torch.tensor(s.pos, dtype=torch.float64, device="cuda")
    ctx = api.Context(0, s.fire, precision="fp64")
    rows = []

    def run(alpha0, tmax, dt):
        r, wall = relax_once(ctx, pos0, s, args.sweep_max_steps, dict(s.fire, alpha0=alpha0, tmax=tmax, dt_start=dt))
        rows.append({"alpha0": alpha0, "tmax": tmax, "dt_ps": dt, "stop": r["stop"], "force_evals": r["force_evals"],
                     "ms": wall * 1e3})
        log(f"[study] alpha0 {alpha0} tmax {tmax} dt {dt * 1e3:.1f} fs: {r['stop']} after {r['force_evals']} evaluations")

    for tmax in (2, 4, 6, 10, 15, 20):
        for alpha0 in (0.05, 0.1, 0.15, 0.2, 0.25, 0.3, 0.4):
            run(alpha0, tmax, 0.001)
    for dt in (0.0005, 0.002, 0.004):
        for tmax in (2, 4, 6, 8, 10, 12, 15, 20):
            run(0.15, tmax, dt)
    ctx.close()
    return {"study": "sweep", "workload": "si_slab", "max_steps": args.sweep_max_steps, "rows": rows}


def study_batched_sweep(args):
    """The parameter study as one batched launch: 512 copies of a 2,042-atom
    EAM-form crystal with a vacancy-rich, noisy start, each relaxed with its own
    (alpha0, tmax, dt) from an 8 x 8 x 8 grid (per-system fire_params), against
    a sample of the same runs through the single-system path."""
    import torch
    from paper_1908_02038_amd import api, inputs
    s = inputs.gupta_box(8, nvac=6, noise=0.08, seed=13)
    alphas = (0.05, 0.1, 0.15, 0.2, 0.25, 0.3, 0.35, 0.4)
    tmaxs = (2, 4, 6, 8, 10, 12, 15, 20)
    dts = (0.0005, 0.001, 0.0015, 0.002, 0.0025, 0.003, 0.0035, 0.004)
    grid = [(a, t, d) for d in dts for t in tmaxs for a in alphas]
    per = [dict(s.fire, alpha0=a, tmax=t, dt_start=d) for a, t, d in grid]
    n = len(s.pos)
    src = torch.tensor(np.concatenate([s.pos] * len(grid)), dtype=torch.float64, device="cuda")
    offs = np.arange(len(grid) + 1, dtype=np.int64) * n
    boxes = [s.box] * len(grid)
    ctx = api.Context(0, s.fire)
    work = src.clone()
    ctx.fire_minimize_batched_dev(work, offs, boxes, s.potential, s.tol, args.sweep_max_steps, per_sys=per)
    work.copy_(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = ctx.fire_minimize_batched_dev(work, offs, boxes, s.potential, s.tol, args.sweep_max_steps, per_sys=per)
    torch.cuda.synchronize()
    dt_batch = time.perf_counter() - t0
    ctx.close()
    # the single-system path on every 32nd grid point
    ctx = api.Context(0, s.fire, precision="fp64")
    pos0 = torch.tensor(s.pos, dtype=torch.float64, device="cuda")
    sample, t_plain, same = list(range(0, len(grid), 32)), 0.0, 0
    for k in sample:
        r, wall = relax_once(ctx, pos0, s, args.sweep_max_steps, per[k])
        t_plain += wall
        same += r["force_evals"] == res[k]["force_evals"]
    ctx.close()
    rows = [{"alpha0": a, "tmax": t, "dt_ps": d, "stop": r["stop"], "force_evals": r["force_evals"]}
            for (a, t, d), r in zip(grid, res)]
    log(f"[study] batched sweep: {len(grid)} relaxations of {n} atoms in {dt_batch * 1e3:.1f} ms; single-system path "
        f"{t_plain / len(sample) * 1e3:.1f} ms per relaxation on {len(sample)} of them "
        f"({same} with the same evaluation count)")
    return {"study": "batched_sweep", "atoms": n, "systems": len(grid), "ms_batch": dt_batch * 1e3,
            "ms_plain_per_relaxation": t_plain / len(sample) * 1e3, "plain_sample": len(sample),
            "plain_same_evals": same, "rows": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="lj_bulk",
                    choices=["lj_small", "lj_bulk", "gupta_bulk", "gupta_slab", "si_slab"])
    ap.add_argument("--max-steps", type=int, default=100000)
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-configs", action="store_true", help="skip the other configurations")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--kernel-reps", type=int, default=50)
    ap.add_argument("--kernel-only", action="store_true",
                    help="only the dominant force pass (reps launches) and a plain copy of known size; "
                         "for hardware-counter runs")
    ap.add_argument("--kernel-precision", choices=["fp64", "mixed", "fp32"], default="fp64",
                    help="pair precision of the --kernel-only passes (mixed starts with FP32 pair terms)")
    ap.add_argument("--study", choices=["integrators", "sweep", "batched_sweep"],
                    help="instead of the bench line: one JSON line of the integrator comparison or the parameter "
                         "sweep")
    ap.add_argument("--sweep-max-steps", type=int, default=20000)
    ap.add_argument("--fp32-max-steps", type=int, default=3000,
                    help="iteration limit of the pure FP32 run (it cannot reach 1e-6)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "the FIRE path runs on one GPU only; --gpus must be 1 "
                          "(a multi-GPU decomposition is designed but not built)"}))
        sys.exit(2)

    import torch
    from paper_1908_02038_amd import api

    assert torch.cuda.is_available(), "bench needs a GPU"
    s = make_system(args.workload)
    n = len(s.pos)
    kind = s.potential["kind"]
    log(f"[bench] workload {args.workload}: {n} atoms, potential {kind}, tol {s.tol}")
    pos0 = torch.tensor(s.pos, dtype=torch.float64, device="cuda")
    if args.kernel_only:
        kernel_only(args, s, pos0)
        return
    if args.study:
        out = {"integrators": study_integrators, "sweep": study_sweep,
               "batched_sweep": study_batched_sweep}[args.study](args)
        print(json.dumps(out), flush=True)
        return

    # ---- FP64 plain path (headline)
    ctx = api.Context(0, s.fire, precision="fp64")
    dt, res, final = time_relaxations(ctx, pos0, s, args.steps, args.warmup, args.max_steps)
    r = res[-1]
    evals = sum(x["force_evals"] for x in res)
    iters = sum(x["iterations"] for x in res)
    value = n * evals / dt
    log(f"[bench] fp64: {args.steps} relaxations in {dt:.3f} s, {r['iterations']} iterations each, "
        f"stop {r['stop']}, E/N {r['energy_per_atom']:.12f}, fmax {r['fmax']:.3e}, rebuilds {r['rebuilds']}")
    kt = kernel_time_ms(ctx, args.kernel_reps)
    # LDS-staged tiles (and the folded update) unless switched off; the
    # three-body path always gathers from global memory
    staged = os.environ.get("FIRE_LDS", "1") != "0" and kind != "sw"
    alg = FUSED[kind] if staged else ALG[kind]
    bytes_launch = alg["bytes"] * n
    flops_launch = alg["flops"] * n
    hbm_ach = bytes_launch / (kt * 1e-3) / 1e9
    alu_ach = flops_launch / (kt * 1e-3) / 1e12
    ridge = PEAK_FP64_TFLOPS * 1e12 / (PEAK_HBM_GBS * 1e9)
    ai = alg["flops"] / alg["bytes"]
    kname = alg["kernel"]
    traffic = load_traffic(alg["tag"], args.workload)
    if ai > ridge:
        roof = {"bound": "alu", "achieved": alu_ach, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": alu_ach / PEAK_FP64_TFLOPS}
    else:
        roof = {"bound": "hbm", "achieved": hbm_ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": hbm_ach / PEAK_HBM_GBS}
    roof.update({"traffic": traffic,
                 "limiter": load_limiter(alg["tag"], args.workload),
                 "kernel": kname if (staged or kind == "sw") else kname + "<double, false, false>",
                 "ms_per_launch": kt,
                 "algorithmic_bytes_per_launch": bytes_launch, "algorithmic_flops_per_launch": flops_launch,
                 "hbm_achieved_GBs": hbm_ach, "hbm_frac": hbm_ach / PEAK_HBM_GBS,
                 "arithmetic_intensity": ai, "ridge": ridge})
    log(f"[bench] force pass {kt * 1e3:.1f} us/launch: {hbm_ach:.0f} GB/s alg ({hbm_ach / PEAK_HBM_GBS:.3f} of HBM), "
        f"{alu_ach:.2f} TFLOP/s alg ({alu_ach / PEAK_FP64_TFLOPS:.3f} of FP64)")
    ctx.close()

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "atom-force-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "atoms": n, "potential": kind, "fmax_tol": s.tol,
                   "fire": {k: s.fire[k] for k in ("dt_start", "tmax", "alpha0", "delaystep", "dtgrow",
                                                   "dtshrink", "integrator")},
                   "neighbour_skin": s.fire.get("skin", "library default: 0.12 x cutoff")},
        "steps_per_s": iters / dt,
        "iterations_per_relaxation": r["iterations"],
        "stop": r["stop"],
        "energy_per_atom": r["energy_per_atom"],
        "fmax": r["fmax"],
        "roofline": roof,
    }

    # ---- mixed precision on the same input
    if not args.no_mixed and kind != "sw":  # the three-body path has no FP32 terms
        ctxm = api.Context(0, s.fire, precision="mixed")
        dtm, resm, _ = time_relaxations(ctxm, pos0, s, args.steps, args.warmup, args.max_steps)
        rm = resm[-1]
        evm = sum(x["force_evals"] for x in resm)
        itm = sum(x["iterations"] for x in resm)
        ktm = kernel_time_ms(ctxm, args.kernel_reps)  # params say mixed -> FP32 pair kernel
        ctxm.close()
        # the FP32 force floor: max |F_i| of FP32 pair terms at the FP64
        # minimum just found (where the FP64 forces are below the tolerance)
        ctx32 = api.Context(0, s.fire, precision="fp32")
        _, f32 = ctx32.fire_energy_forces_dev(final, s.box, s.potential)
        floor = float(torch.linalg.norm(f32, dim=1).max())
        # the pure FP32 path (no switch to FP64 pair terms) toward the same tolerance
        w32 = pos0.clone()
        r32 = ctx32.fire_minimize_dev(w32, s.box, s.potential, s.tol, args.fp32_max_steps)
        ctx32.close()
        out["mixed"] = {
            "value": n * evm / dtm,
            "ms_per_step": dtm / args.steps * 1e3,
            "steps_per_s": itm / dtm,
            "iterations_per_relaxation": rm["iterations"],
            "iterations_fp32": rm["iterations_low"],
            "stop": rm["stop"],
            "energy_per_atom": rm["energy_per_atom"],
            "energy_per_atom_rel_diff_vs_fp64": abs(rm["energy_per_atom"] - r["energy_per_atom"])
            / abs(r["energy_per_atom"]),
            "fmax": rm["fmax"],
            "fp32_force_pass_ms": ktm,
            "fp32_force_pass_kernel": FP32_KERNEL.get(kind, ""),
            "speedup_vs_fp64_wall": dt / args.steps / (dtm / args.steps),
            "fp32_force_floor": floor,
            "fp32_force_floor_note": "max |F_i| of FP32 pair terms at the FP64 path's relaxed positions",
            "pure_fp32": {"stop": r32["stop"], "iterations": r32["iterations"], "fmax": r32["fmax"],
                          "energy_per_atom": r32["energy_per_atom"],
                          "energy_per_atom_rel_diff_vs_fp64": abs(r32["energy_per_atom"] - r["energy_per_atom"])
                          / abs(r["energy_per_atom"]),
                          "max_steps": args.fp32_max_steps},
        }
        log(f"[bench] mixed: {rm['iterations']} iterations ({rm['iterations_low']} FP32), "
            f"{dtm / args.steps * 1e3:.1f} ms/relaxation, FP32 force pass {ktm * 1e3:.1f} us; FP32 force floor "
            f"{floor:.3e}; pure FP32: {r32['stop']} after {r32['iterations']} iterations, fmax {r32['fmax']:.3e}")

    if not args.no_batched:
        out["batched"] = bench_batched(args)

    if not args.no_configs and args.workload == "lj_bulk":
        out["other_configs"] = other_configs(args)

    if not args.no_cpu:
        log("[bench] cpu oracle baseline ...")
        out["cpu_baseline"] = cpu_baseline(s, args.cpu_budget)
        log(f"[bench] cpu: {out['cpu_baseline']['sample']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
