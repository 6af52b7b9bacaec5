#!/usr/bin/env python3
"""Throughput of the D2Q9 lattice-Boltzmann hot path on one MI355X.

Workload (precision-and-batching stress): one 8192x8192 periodic domain plus
200 uneven periodic domains of 64^2..2048^2 (log-uniform sides, RSA disc
obstacles at 20% solid, tau ~ U[0.55, 1.2]), all started from seeded shear
waves (u0 = 0.01).  Every step advances all 201 domains with one sweep launch
(batched, replayed from a hipGraph).  Populations are stored as FP16 deviations
with stochastic rounding (the reported value), and, for comparison, as plain
FP32 and as BF16 deviations; arithmetic is FP32.  Each launch of the
two-step sweep advances every domain by two steps; before the timed region
lb_batch_autotune picks its tile height (timed once per process, then
cached).  With --single-step (one step per launch) the single-step tile
shapes are tuned instead, on a throwaway copy of the batch.  The first call
captures every step graph the timed calls replay.

MLUPS counts every lattice site of every domain (solids included), as the
paper defines it.  The roofline object reports the sweep kernel's algorithmic
HBM bytes per launch over its measured average launch duration against 8 TB/s
(HIP events on the launch stream; the duration is the difference between a
call of 2K steps and the timed call of K steps, which removes each call's
fixed cost, the FP64 density sums).  The CPU baseline is the FP64 oracle on a
bounded sample of the smallest domains of the same workload, 1000 steps each,
on all host threads the process may use (at most 16) and on one thread, and on
a few steps of each other workload's lattice; the same sample, run on the GPU
for 1000 steps in each storage format, gives the relative L2 velocity error
against the oracle (the workload's stated horizon), whatever --steps is.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "MLUPS and % of HBM roofline, FP16-delta batched vs plain FP32 at stated L2 error"
BIG_N = 8192
ACC_STEPS = 1000   # horizon of the L2 comparison against the oracle
L2_TARGET = {"f32": 1e-5, "f16": 1e-3, "bf16": 1e-3}
BIG_TAU = 0.8
N_SMALL = 200
SHEAR_U0 = 0.01
STORAGE_BYTES = {"f16": 2, "bf16": 2, "f32": 4}
ROUNDING = {"f16": "stochastic", "bf16": "stochastic", "f32": "nearest"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_traffic.json")
SWEEP_SOURCES = ["paper_2006_12910_amd/csrc/sweep_impl.h", "paper_2006_12910_amd/csrc/sweep2_impl.h",
                 "paper_2006_12910_amd/csrc/lb_device.h", "paper_2006_12910_amd/csrc/kernels_st.h",
                 "paper_2006_12910_amd/csrc/lb_api.hip", "paper_2006_12910_amd/build.py"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def sweep_source_hash():
    h = hashlib.sha256()
    for rel in SWEEP_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def workload():
    from paper_2006_12910_amd import inputs
    specs = [dict(n=BIG_N, tau=BIG_TAU, k=1, phase=0.0, obstacle_seed=None)]
    specs += inputs.stress_batch(count=N_SMALL, seed=0)
    return specs


def domain_inputs(spec):
    from paper_2006_12910_amd import inputs
    n = spec["n"]
    fields = inputs.shear_wave_field(n, n, SHEAR_U0, spec["k"], spec["phase"])
    mask = None if spec["obstacle_seed"] is None else inputs.stress_obstacles(n, spec["obstacle_seed"])
    return fields, mask


def size_bucket(spec):
    """(has obstacles, size class); the class edges 128 and 256 are those of
    the library's default tile widths, so a class shares one default shape."""
    n = spec["n"]
    return (spec["obstacle_seed"] is not None,
            0 if n < 128 else 1 if n < 256 else 2 if n < 1024 else 3 if n < 4096 else 4)


def autotune_tiles(storage, specs, masks):
    """Tile shape per size class: lb_autotune (every tile width and rows per
    thread, timed with HIP events) on a throwaway copy of the largest member
    of each class with sides of 1024 or more; the batch members of the class
    then take its choice (smaller classes keep the default shape)."""
    from paper_2006_12910_amd import lb
    best = {}
    for b in sorted({size_bucket(s) for s in specs}):
        i = max((j for j, s in enumerate(specs) if size_bucket(s) == b), key=lambda j: specs[j]["n"])
        n = specs[i]["n"]
        if n < 1024:
            continue  # a step of a small domain is too short to time: default shape
        d = lb.Domain(n, n, tau=specs[i]["tau"], storage=storage, rounding=ROUNDING[storage],
                      obstacles=masks[i])
        ms = d.autotune(steps=10 if n >= 2048 else 40)
        best[b] = (d.get_option(lb.OPT_TILE_WIDTH), d.get_option(lb.OPT_ROWS_PER_THREAD))
        log(f"{storage}: autotune class {b} ({n}^2): tile {best[b][0]}x{best[b][1]}, {ms * 1e3:.1f} us/step")
        d.close()
    return best


def tune_batch(storage, specs, masks, steps=20):
    """Tile shape of every batch member, chosen by timing the batch step itself
    (HIP events, on a throwaway copy of the batch) for the library's default
    shapes, for every uniform shape, and for lb_autotune's per-class shapes;
    returns the fastest assignment {class: (tile_w, rows)}, None = defaults."""
    import torch
    from paper_2006_12910_amd import lb
    classes = sorted({size_bucket(s) for s in specs})
    cands = [("defaults", None)]
    cands += [(f"uniform {tw}x{r}", {c: (tw, r) for c in classes}) for tw in (64, 128, 256) for r in (2, 4, 8)]
    cands.append(("per-class autotune", autotune_tiles(storage, specs, masks)))
    doms = build_variant(storage, specs, masks)
    for d in doms:
        d.set_option(lb.OPT_TWO_STEP, 0)  # the shapes tuned are the single-step sweep's
    default = [(d.get_option(lb.OPT_TILE_WIDTH), d.get_option(lb.OPT_ROWS_PER_THREAD)) for d in doms]
    stream = torch.cuda.current_stream()
    best = None
    for name, tiles in cands:
        for d, spec, dflt in zip(doms, specs, default):
            tw, rows = tiles[size_bucket(spec)] if tiles and size_bucket(spec) in tiles else dflt
            d.set_option(lb.OPT_TILE_WIDTH, tw)
            d.set_option(lb.OPT_ROWS_PER_THREAD, rows)
        batch = lb.Batch(doms)
        batch.step(3)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        batch.step(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        batch.close()
        log(f"{storage}: batch tuning, {name}: {ms:.3f} ms/step")
        if best is None or ms < best[0]:
            best = (ms, name, tiles)
    for d in doms:
        d.close()
    torch.cuda.empty_cache()
    log(f"{storage}: batch tuning chose {best[1]}")
    return best[2]


def build_variant(storage, specs, masks, tiles=None):
    from paper_2006_12910_amd import lb
    doms = []
    for i, spec in enumerate(specs):
        fields, _ = domain_inputs(dict(spec, obstacle_seed=None))
        d = lb.Domain(spec["n"], spec["n"], tau=spec["tau"], storage=storage,
                      rounding=ROUNDING[storage], init=fields, obstacles=masks[i])
        if tiles and size_bucket(spec) in tiles:
            tw, rows = tiles[size_bucket(spec)]
            d.set_option(lb.OPT_TILE_WIDTH, tw)
            d.set_option(lb.OPT_ROWS_PER_THREAD, rows)
        doms.append(d)
    return doms


def algorithmic_bytes(specs, masks, sbytes):
    """Bytes the sweep must move per step: 9 loads + 9 stores of each fluid
    node's populations, plus the 2-byte node word (solid flag and solid-source
    mask) of every site of a domain with obstacles."""
    total = 0
    for spec, m in zip(specs, masks):
        n2 = spec["n"] * spec["n"]
        fluid = n2 if m is None else n2 - int(m.sum())
        total += 18 * sbytes * fluid + (0 if m is None else 2 * n2)
    return total


def parse_tiles(text):
    """{"open/class3": "64x4", ...} (the "tiles" object of a bench line) ->
    {(False, 3): (64, 4), ...}"""
    out = {}
    for k, v in json.loads(text).items():
        kind, cls = k.split("/class")
        tw, rows = v.split("x")
        out[(kind == "obstacles", int(cls))] = (int(tw), int(rows))
    return out


def timed_call(batch, steps):
    """ms of one lb_batch_step(steps) call: HIP events on the batch's stream
    (the stream the sweep is launched on)."""
    import torch
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    batch.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def run_variant(storage, specs, masks, steps, warmup, tune, fixed_tiles=None, two_step=True):
    """The batch of the workload in one storage format, timed over `steps`
    steps after `warmup` (the first call captures every step graph the batch
    uses, so nothing is captured inside the timed call).  With single steps
    the autotuner picks the members' tile shapes.  Also
    returns the ms of a following call of 2 * steps steps.  An untimed call
    of `steps` steps precedes the timed one.  With the two-step sweep the
    batch's tile height comes from lb_batch_autotune (unless --no-tune)."""
    import torch
    from paper_2006_12910_amd import lb
    t0 = time.time()
    tiles = fixed_tiles if fixed_tiles else (
        tune_batch(storage, specs, masks) if tune and not two_step else None)
    doms = build_variant(storage, specs, masks, tiles)
    for d in doms:
        d.set_option(lb.OPT_TWO_STEP, 1 if two_step else 0)
    # the single-step shapes in use, per class (explicit also where the
    # defaults won)
    tiles = None
    if not two_step:
        tiles = {}
        for d, spec in zip(doms, specs):
            tiles.setdefault(size_bucket(spec), (d.get_option(lb.OPT_TILE_WIDTH),
                                                 d.get_option(lb.OPT_ROWS_PER_THREAD)))
    batch = lb.Batch(doms)
    torch.cuda.synchronize()
    log(f"{storage}: built {len(doms)} domains in {time.time() - t0:.1f}s")
    if two_step and tune:
        # the two-step tile height: lb_batch_autotune (timed, or from its cache)
        ms_t = batch.autotune(steps=16)
        log(f"{storage}: batch two-step tile height {batch.get_option(lb.OPT_TWO_STEP_ROWS)} "
            f"({'timed, ' + format(ms_t, '.3f') + ' ms/step' if ms_t > 0 else 'cached'})")
    batch.step(max(warmup, 1))
    # one untimed call of the timed length first (a 20-step call timed right
    # after a 5-step warm-up took ~3 ms more than its share of a 40-step call)
    batch.step(steps)
    torch.cuda.synchronize()
    ms = timed_call(batch, steps)
    log(f"{storage}: {steps} steps in {ms:.1f} ms")
    ms2 = timed_call(batch, 2 * steps)
    log(f"{storage}: {2 * steps} steps in {ms2:.1f} ms")
    if two_step:
        tiles = f"two-step: 62 columns x {batch.get_option(lb.OPT_TWO_STEP_ROWS)} rows per tile" + (
            " (lb_batch_autotune)" if tune else " (default)")
    return doms, batch, ms, ms2, tiles


def run_oracle(specs, masks, nsteps, budget_s):
    """The oracle on the smallest domains of the workload, in order of size,
    until its stepping time reaches the budget: returns the final moments of
    each domain it ran, its MLUPS and its stepping time."""
    from oracle import Oracle, OracleParams
    results, t_total, sites = {}, 0.0, 0
    for i in sorted(range(len(specs)), key=lambda k: specs[k]["n"]):
        if t_total >= budget_s:
            break
        spec = specs[i]
        n = spec["n"]
        fields, _ = domain_inputs(dict(spec, obstacle_seed=None))
        o = Oracle(OracleParams(nx=n, ny=n, tau=spec["tau"]), masks[i], *fields)
        t0 = time.perf_counter()
        o.run(nsteps)
        t_total += time.perf_counter() - t0
        sites += n * n * nsteps
        results[i] = o.moments()
    return results, sites / t_total / 1e6, t_total


def cpu_baseline_leg(specs, masks, args):
    """The CPU baseline: the oracle on the smallest domains of the workload
    (all host threads up to 16, then one thread), and, unless the other
    workloads are skipped, on each of them.  Returns the cpu_baseline entry
    and the sample's final moments (the reference of the accuracy leg)."""
    threads = min(len(os.sched_getaffinity(0)), 16)
    os.environ["OMP_NUM_THREADS"] = str(threads)
    ref, cpu_mlups, cpu_s = run_oracle(specs, masks, ACC_STEPS, args.cpu_budget)
    sample = sorted(ref)
    set_omp_threads(1)
    _, cpu1_mlups, cpu1_s = run_oracle(specs, masks, ACC_STEPS, args.cpu_budget / 3)
    set_omp_threads(threads)
    cpu = {"value": round(cpu_mlups, 2), "unit": "MLUPS", "cores": threads, "kind": "oracle",
           "sample": f"{len(sample)} smallest domains of the workload "
                     f"({min(specs[i]['n'] for i in sample)}^2..{max(specs[i]['n'] for i in sample)}^2), "
                     f"{ACC_STEPS} steps each, FP64, {cpu_s:.1f}s",
           "cpu_model": cpu_model(), "host_threads_visible": len(os.sched_getaffinity(0)),
           "one_thread_value": round(cpu1_mlups, 2),
           "one_thread_sample": f"smallest domains in order, {ACC_STEPS} steps each, {cpu1_s:.1f}s"}
    log(f"oracle: {cpu_mlups:.2f} MLUPS on {threads} threads, {len(sample)} domains; "
        f"{cpu1_mlups:.2f} MLUPS on one thread ({cpu_model()})")
    if not args.no_configs:
        t0 = time.time()
        cpu["other_workloads"] = cpu_baseline_other_workloads()
        log(f"oracle on the other workloads ({time.time() - t0:.0f}s): {json.dumps(cpu['other_workloads'])}")
    return cpu, ref


def set_omp_threads(n):
    """Thread count of the oracle's OpenMP loops (process-wide libgomp)."""
    import ctypes
    ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def accuracy_leg(storage, specs, masks, ref):
    """The oracle's sample domains on the GPU in `storage`, batched as in the
    timed run, advanced ACC_STEPS steps: relative L2 velocity errors."""
    from paper_2006_12910_amd import lb
    idx = sorted(ref)
    sub = [specs[i] for i in idx]
    doms = build_variant(storage, sub, [masks[i] for i in idx])
    batch = lb.Batch(doms)
    batch.step(ACC_STEPS)
    out = l2_errors({i: d for i, d in zip(idx, doms)}, ref)
    batch.close()
    for d in doms:
        d.close()
    tgt = L2_TARGET[storage]
    out.update(after_steps=ACC_STEPS, domains=len(idx), target=tgt,
               target_met_vs_u_T=out["max_vs_u_T"] <= tgt, target_met_vs_u_0=out["max_vs_u_0"] <= tgt)
    return out


def l2_errors(doms, ref):
    errs_t, errs_0 = [], []
    for i, (r, u, v) in ref.items():
        rg, ug, vg = doms[i].moments()
        num = np.sqrt(((ug - u) ** 2 + (vg - v) ** 2).sum())
        errs_t.append(num / np.sqrt((u ** 2 + v ** 2).sum()))
        fluid = r > 0
        errs_0.append(num / (SHEAR_U0 * np.sqrt(0.5 * fluid.sum())))  # |u(0)| over fluid sites
    return dict(max_vs_u_T=float(np.max(errs_t)), median_vs_u_T=float(np.median(errs_t)),
                max_vs_u_0=float(np.max(errs_0)), median_vs_u_0=float(np.median(errs_0)))


def copy_bandwidth(mib=2048, reps=10):
    """Measured device-to-device copy rate (1:1 read/write, like the sweep)."""
    import torch
    a = torch.empty(mib << 20, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * a.numel() * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbs


def other_configs():
    """GPU MLUPS of the other four workloads, of the 8192^2 member alone and
    of the D3Q19 and D3Q27 lattices at their full sizes (timed with HIP events after a
    warm-up call); the oracle's rates on the same lattices are part of the
    CPU baseline."""
    import torch
    from paper_2006_12910_amd import inputs, lb
    out = {}

    def gpu_rate(name, dom_or_batch, sites, steps):
        dom_or_batch.step(max(steps // 10, 1))
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dom_or_batch.step(steps)
        e1.record()
        torch.cuda.synchronize()
        out[name] = {"gpu_mlups": round(sites * steps / (e0.elapsed_time(e1) * 1e-3) / 1e6, 1)}

    # a single-domain probe above 1 GB: the 8192^2 periodic shear wave alone,
    # FP16 deviations with stochastic rounding, two steps per launch
    # (algorithmic bytes 36 per site update; the A-B buffers take 2.4 GB)
    fields = inputs.shear_wave_field(8192, 8192, SHEAR_U0, 1, 0.0)
    d = lb.Domain(8192, 8192, tau=BIG_TAU, storage="f16", rounding="stochastic", init=fields)
    del fields
    gpu_rate("single_8192_f16", d, 8192 * 8192, 200)
    d.close()
    r = out["single_8192_f16"]
    r["sweep_GBps"] = round(r["gpu_mlups"] * 1e6 * 36 / 1e9, 1)
    r["hbm_frac"] = round(r["sweep_GBps"] / HBM_PEAK_GBS, 4)
    torch.cuda.empty_cache()
    # channel 128 x 64, FP64
    kw = dict(bc_y="wall", tau=0.8, g=(1e-6, 0.0))
    d = lb.Domain(128, 64, storage="f64", **kw)
    gpu_rate("channel_128x64_f64", d, 128 * 64, 5000)
    d.close()
    # porous 2048 x 1024 with 16 discs, FP32 storage
    mask, _ = inputs.porous_channel()
    parts = [dict(x=x, y=y, radius=8.0, density_ratio=1.05) for x, y in inputs.particle_block()]
    lj = (1e-3, 2.5, 0.5)
    d = lb.Domain(2048, 1024, storage="f32", bc_x="pressure", bc_y="wall", tau=0.7, rho_in=1.001,
                  rho_out=0.999, obstacles=mask, max_particles=16, lj=lj)
    d.set_option(lb.OPT_FORCE_AVERAGE, 1)
    d.add_particles(parts)
    gpu_rate("porous_2048x1024_16discs_f32", d, 2048 * 1024, 1000)
    # the same with the particle coupling overlapping the bulk sweep
    d.set_option(lb.OPT_OVERLAP, 1)
    gpu_rate("porous_2048x1024_16discs_f32_overlapped", d, 2048 * 1024, 1000)
    d.close()
    # fluctuating 512^2 with a Brownian disc, FP32 storage; and the 64-member ensemble
    d = lb.Domain(512, 512, storage="f32", tau=1.0, kT=1e-4, seed=2006, domain_id=1, max_particles=1)
    d.add_particles([dict(x=256.5, y=256.5, radius=5.0)])
    gpu_rate("fluctuating_512_disc_f32", d, 512 * 512, 2000)
    d.close()
    # the 64-member ensemble in FP32 and in FP16 deviations (stochastic rounding)
    for storage in ("f32", "f16"):
        b, doms, sites = fluct_ensemble(storage)
        gpu_rate(f"fluctuating_ensemble_64_{storage}", b, sites, 200)
        b.close()
        for dd in doms:
            dd.close()
    # power-law channel 4096 x 256, n = 0.5, FP32 storage
    d, _, _ = powerlaw_channel("f32")
    gpu_rate("powerlaw_4096x256_n0.5_f32", d, 4096 * 256, 2000)
    d.close()
    # the 3D lattices: 256^3 periodic, one sweep per step, FP32 storage and
    # FP16 deviations (stochastic rounding); algorithmic bytes 2 q s per node
    # update (q = 19 or 27, s = 4 or 2)
    n3 = 256
    for lattice, q in (("d3q19", 19), ("d3q27", 27)):
        for storage, sb in (("f32", 4), ("f16", 2)):
            d, _, _ = d3q19_cube(storage, n3, lattice)
            name = f"{lattice}_256cube_{storage}"
            gpu_rate(name, d, n3 ** 3, 200)
            d.close()
            r = out[name]
            r["sweep_GBps"] = round(r["gpu_mlups"] * 1e6 * 2 * q * sb / 1e9, 1)
            r["hbm_frac"] = round(r["sweep_GBps"] / HBM_PEAK_GBS, 4)
        # with thermal noise, kT = 1e-4 (q normals a node: Philox blocks and
        # Box-Muller pairs in the sweep)
        for storage, sb in (("f32", 4), ("f16", 2)):
            d, _, _ = d3q19_cube(storage, n3, lattice, kT=1e-4)
            name = f"{lattice}_256cube_{storage}_noise"
            gpu_rate(name, d, n3 ** 3, 200)
            d.close()
            r = out[name]
            r["sweep_GBps"] = round(r["gpu_mlups"] * 1e6 * 2 * q * sb / 1e9, 1)
            r["hbm_frac"] = round(r["sweep_GBps"] / HBM_PEAK_GBS, 4)
    torch.cuda.empty_cache()
    return out


def fluct_ensemble(storage="f32"):
    """The batched fluctuating workload: 64 realisations of 128^2..1024^2,
    each with a Brownian disc of radius 5, kT = 1e-4, tau = 1 (16-bit
    storage with stochastic rounding)."""
    from paper_2006_12910_amd import inputs, lb
    specs = inputs.fluctuating_batch(count=64)
    doms = []
    for sp in specs:
        dd = lb.Domain(sp["n"], sp["n"], storage=storage, tau=1.0, kT=1e-4, seed=64,
                       domain_id=sp["domain_id"], max_particles=1, rounding=ROUNDING[storage])
        cx, cy, r = sp["disc"]
        dd.add_particles([dict(x=cx, y=cy, radius=r)])
        doms.append(dd)
    return lb.Batch(doms), doms, sum(sp["n"] ** 2 for sp in specs)


def porous_discs(storage="f32"):
    """Porous 2048 x 1024 (35 % discs, density faces) with 16 mobile discs."""
    from paper_2006_12910_amd import inputs, lb
    mask, _ = inputs.porous_channel()
    parts = [dict(x=x, y=y, radius=8.0, density_ratio=1.05) for x, y in inputs.particle_block()]
    d = lb.Domain(2048, 1024, storage=storage, bc_x="pressure", bc_y="wall", tau=0.7, rho_in=1.001,
                  rho_out=0.999, obstacles=mask, max_particles=16, lj=(1e-3, 2.5, 0.5))
    d.set_option(lb.OPT_FORCE_AVERAGE, 1)
    d.add_particles(parts)
    return d, [d], 2048 * 1024


def powerlaw_channel(storage="f32"):
    """Power-law channel 4096 x 256, n = 0.5, K = 0.01, tau* in [0.51, 2.5]."""
    from paper_2006_12910_amd import lb
    pl = dict(n=0.5, K=0.01, tau_min=0.51, tau_max=2.5)
    d = lb.Domain(4096, 256, storage=storage, bc_y="wall", g=(2.648e-6, 0.0), power_law=pl)
    return d, [d], 4096 * 256


def d3q19_cube(storage="f32", n=256, lattice="d3q19", kT=0.0):
    """The 3D lattice (D3Q19, or D3Q27): 256^3 periodic, tau = 0.8, at rest
    (16-bit storage with stochastic rounding); kT > 0: thermal noise."""
    from paper_2006_12910_amd import lb
    d = lb.Domain3(n, n, n, tau=0.8, storage=storage, seed=3, lattice=lattice, kT=kT)
    return d, [d], n ** 3


def only_workload(name, steps, warmup):
    """One workload alone (for profiling): warm-up, then `steps` timed steps;
    prints one JSON line."""
    import torch
    make = {"fluct-ensemble": fluct_ensemble, "fluct-ensemble-f16": lambda: fluct_ensemble("f16"),
            "porous": porous_discs, "powerlaw": powerlaw_channel, "d3q19": d3q19_cube,
            "d3q19-f16": lambda: d3q19_cube("f16"),
            "d3q27": lambda: d3q19_cube("f32", lattice="d3q27"),
            "d3q27-f16": lambda: d3q19_cube("f16", lattice="d3q27"),
            "d3q19-noise": lambda: d3q19_cube("f32", kT=1e-4),
            "d3q19-f16-noise": lambda: d3q19_cube("f16", kT=1e-4),
            "d3q27-noise": lambda: d3q19_cube("f32", lattice="d3q27", kT=1e-4)}[name]
    runner, doms, sites = make()
    runner.step(max(warmup, 1))
    torch.cuda.synchronize()
    ms = timed_call(runner, steps)
    print(json.dumps({"workload": name, "steps": steps, "ms_per_step": round(ms / steps, 5),
                      "mlups": round(sites * steps / (ms * 1e-3) / 1e6, 1)}), flush=True)
    if runner is not doms[0]:
        runner.close()
    for d in doms:
        d.close()


# The paper's best CPU rates of its three timing benchmarks (MLUPS, its table
# of optimisation stages: OpenMP with thread affinity, 28-core Xeon E5-2697 v3).
PAPER_BEST_CPU_MLUPS = {"b1": 47.27, "b2": 138.20, "b3": 85.85}


def reporting_offload(steps=600, intervals=(10, 100)):
    """Steps with the moments reported to the host every `interval` steps, on
    the porous 2048 x 1024 workload with 16 discs (FP32): no reporting; the
    synchronous call (lb_moments into pageable host arrays); the offloaded one
    (lb_moments_async on a copy stream into pinned host arrays, two staging
    sets used in turn, each report consumed on the host after its wait while
    later steps run).  Wall-clock ms per step, whole loop synchronised."""
    import numpy as np
    import torch
    from paper_2006_12910_amd import inputs, lb
    mask, _ = inputs.porous_channel()
    parts = [dict(x=x, y=y, radius=8.0, density_ratio=1.05) for x, y in inputs.particle_block()]
    d = lb.Domain(2048, 1024, storage="f32", bc_x="pressure", bc_y="wall", tau=0.7, rho_in=1.001,
                  rho_out=0.999, obstacles=mask, max_particles=16, lj=(1e-3, 2.5, 0.5))
    d.set_option(lb.OPT_FORCE_AVERAGE, 1)
    d.add_particles(parts)
    n = d.nx * d.ny
    copy = torch.cuda.Stream()
    stages = [torch.empty(3 * n, dtype=torch.float64, device="cuda") for _ in range(2)]
    hosts = [[torch.empty((d.ny, d.nx), dtype=torch.float64, pin_memory=True) for _ in range(3)]
             for _ in range(2)]
    sink = []

    def timed(body):
        d.step(20)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        body()
        torch.cuda.synchronize()
        return round((time.perf_counter() - t0) * 1e3 / steps, 4)

    def plain():
        d.step(steps)

    out = {"workload": "porous 2048x1024, 16 discs, FP32", "steps": steps,
           "ms_per_step_no_reporting": timed(plain)}
    for every in intervals:
        def sync():
            for _ in range(steps // every):
                d.step(every)
                r, u, v = d.moments()
                sink.append(float(u[::64, ::64].sum()))

        def offload():
            k = 0
            for _ in range(steps // every):
                d.step(every)
                d.moments_wait()  # the report before last has landed: consume it
                if k >= 1:
                    sink.append(float(hosts[(k - 1) % 2][1].numpy()[::64, ::64].sum()))
                d.moments_async(stages[k % 2], *hosts[k % 2], copy)
                k += 1
            d.moments_wait()
            sink.append(float(hosts[(k - 1) % 2][1].numpy()[::64, ::64].sum()))

        out[f"every_{every}"] = {"sync_ms_per_step": timed(sync),
                                 "offload_ms_per_step": timed(offload)}
    d.close()
    return out


def paper_replicas():
    """GPU MLUPS of stand-ins for the paper's three timing benchmarks on their
    full lattices (FP32 storage; the set-ups of tests/test_gpu_paper_benchmarks.py),
    next to the paper's best CPU figure, which is context only (the oracle's
    rates on the same set-ups are part of the CPU baseline)."""
    import torch
    from paper_2006_12910_amd import inputs, lb
    out = {}

    def rate(name, make_gpu, sites, steps):
        d = make_gpu()
        d.step(max(steps // 10, 1))
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        d.step(steps)
        e1.record()
        torch.cuda.synchronize()
        d.close()
        out[name] = {"gpu_mlups": round(sites * steps / (e0.elapsed_time(e1) * 1e-3) / 1e6, 1),
                     "paper_best_cpu_mlups": PAPER_BEST_CPU_MLUPS[name]}

    mask, centres = inputs.replica_b1()

    def b1_gpu():
        d = lb.Domain(1020, 1620, storage="f32", bc_x="wall", tau=0.636, g=(1e-6, -1e-5),
                      obstacles=mask, max_particles=45, lj=(20.0, 2.5, 0.1))
        d.set_option(lb.OPT_FORCE_AVERAGE, 1)
        d.add_particles([dict(x=x, y=y, radius=6.5) for x, y in centres])
        return d

    rate("b1", b1_gpu, 1020 * 1620, 1000)
    ((bx, by),) = inputs.replica_b2()

    def b2_gpu():
        d = lb.Domain(3000, 41, storage="f32", bc_y="wall", tau=0.8, kT=5e-5, seed=2020,
                      domain_id=2, max_particles=1)
        d.add_particles([dict(x=bx, y=by, radius=7.5)])
        return d

    rate("b2", b2_gpu, 3000 * 41, 5000)
    pl = dict(n=0.5, K=1e-3, tau_min=0.50003, tau_max=0.8)
    rate("b3", lambda: lb.Domain(101, 51, storage="f32", bc_y="wall", tau=0.8, g=(1e-6, 0.0),
                                 power_law=pl),
         101 * 51, 20000)
    torch.cuda.empty_cache()
    return out


def cpu_baseline_other_workloads():
    """CPU-baseline leg for the other workloads: the oracle's MLUPS (all
    host threads up to 16) on a few steps of each lattice that other_configs
    and paper_replicas time on the GPU (the 3D lattices on 64^3 instead of 256^3)."""
    from paper_2006_12910_amd import inputs
    from oracle import Oracle, OracleParams
    from oracle.oracle import PRESSURE, WALL, Oracle3
    out = {}

    def rate(name, ora, sites, steps, **extra):
        t0 = time.perf_counter()
        ora.run(steps)
        out[name] = dict(oracle_mlups=round(sites * steps / (time.perf_counter() - t0) / 1e6, 2), **extra)

    rate("channel_128x64_f64", Oracle(OracleParams(nx=128, ny=64, bc_y=WALL, tau=0.8, gx=1e-6)),
         128 * 64, 2000)
    mask, _ = inputs.porous_channel()
    o = Oracle(OracleParams(nx=2048, ny=1024, bc_x=PRESSURE, bc_y=WALL, tau=0.7, rho_in=1.001,
                            rho_out=0.999, lj_psi=1e-3, lj_rit=2.5, lj_floor=0.5,
                            force_average=True), mask)
    for x, y in inputs.particle_block():
        o.add_particle(x, y, 8.0, 1.05, 0.0, 0.0, 0.0)
    rate("porous_2048x1024_16discs_f32", o, 2048 * 1024, 20)
    o = Oracle(OracleParams(nx=512, ny=512, tau=1.0, kT=1e-4, seed=2006, domain_id=1))
    o.add_particle(256.5, 256.5, 5.0, 1.0, 0.0, 0.0, 0.0)
    rate("fluctuating_512_disc_f32", o, 512 * 512, 100)
    rate("powerlaw_4096x256_n0.5_f32",
         Oracle(OracleParams(nx=4096, ny=256, bc_y=WALL, gx=2.648e-6, power_law=True, n_index=0.5,
                             K=0.01)), 4096 * 256, 20)
    rate("d3q19_256cube_f32", Oracle3(64, 64, 64, tau=0.8), 64 ** 3, 10, oracle_lattice="64^3")
    rate("d3q27_256cube_f32", Oracle3(64, 64, 64, tau=0.8, lattice="d3q27"), 64 ** 3, 10,
         oracle_lattice="64^3")
    mask, centres = inputs.replica_b1()
    o = Oracle(OracleParams(nx=1020, ny=1620, bc_x=WALL, tau=0.636, gx=1e-6, gy=-1e-5,
                            force_average=True), mask)
    for x, y in centres:
        o.add_particle(x, y, 6.5, 1.0, 0.0, 0.0, 0.0)
    rate("b1", o, 1020 * 1620, 10)
    ((bx, by),) = inputs.replica_b2()
    o = Oracle(OracleParams(nx=3000, ny=41, bc_y=WALL, tau=0.8, kT=5e-5, seed=2020, domain_id=2))
    o.add_particle(bx, by, 7.5, 1.0, 0.0, 0.0, 0.0)
    rate("b2", o, 3000 * 41, 100)
    rate("b3", Oracle(OracleParams(nx=101, ny=51, bc_y=WALL, tau=0.8, gx=1e-6, power_law=True,
                                   n_index=0.5, K=1e-3, tau_min=0.50003, tau_max=0.8)),
         101 * 51, 2000)
    return out


def profile_entry(steps_per_launch):
    """The dominant sweep kernel's profile (profiles/), or None if the sweep
    sources changed since or the profile covers another kernel."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        t = json.load(fh)
    if t.get("sweep_source_hash") != sweep_source_hash():
        return None
    if t.get("steps_per_launch", 1) != steps_per_launch:
        return None
    return t


def traffic_entry(steps_per_launch):
    """Measured HBM bytes per launch of the dominant sweep kernel, or None."""
    t = profile_entry(steps_per_launch)
    return None if t is None else t.get("hbm_bytes_per_launch")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=900)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--variants", default="f16,f32,bf16",
                    help="storage formats to run; the first is the reported value")
    ap.add_argument("--cpu-budget", type=float, default=15.0,
                    help="seconds of oracle work for the CPU baseline and the L2 sample")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU baseline and L2 sample")
    ap.add_argument("--no-tune", action="store_true", help="default tile shapes instead of the autotuner's")
    ap.add_argument("--single-step", action="store_true",
                    help="one step per launch (two-step sweep off), tile shapes autotuned")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the rates of the other four workloads and of the paper's three "
                         "benchmarks (reported beside the main line)")
    ap.add_argument("--tiles", default=None, metavar="JSON",
                    help='tile shape per size class instead of tuning, e.g. the "tiles" object of an '
                         'earlier line (to profile the configuration that line measured)')
    ap.add_argument("--only", default=None,
                    choices=["fluct-ensemble", "fluct-ensemble-f16", "porous", "powerlaw", "d3q19",
                             "d3q19-f16", "d3q27", "d3q27-f16", "d3q19-noise",
                             "d3q19-f16-noise", "d3q27-noise"],
                    help="time one other workload alone (GPU only; for profiling) and exit")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MiB",
                    help="before the workload, copy a buffer of this size 5 times (a kernel of "
                         "known traffic for scaling profiler byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the domains of a batch would shard across GPUs with no communication).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2006_12910_amd import lb
    assert torch.cuda.is_available(), "bench.py needs an MI355X"
    variants = [v.strip() for v in args.variants.split(",") if v.strip()]
    if args.calibrate_copy > 0:
        a = torch.empty(args.calibrate_copy << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"calibration copy: 5 x {args.calibrate_copy} MiB")
        del a, b
        torch.cuda.empty_cache()
    if args.only:
        only_workload(args.only, args.steps, args.warmup)
        return
    specs = workload()
    t0 = time.time()
    masks = [None if s["obstacle_seed"] is None else domain_inputs(s)[1] for s in specs]
    log(f"inputs: {len(specs)} domains, {sum(s['n'] ** 2 for s in specs) / 1e6:.1f} M sites "
        f"({time.time() - t0:.1f}s)")
    sites = sum(s["n"] ** 2 for s in specs)
    fluid_sites = sum(s["n"] ** 2 - (0 if m is None else int(m.sum())) for s, m in zip(specs, masks))

    ref, cpu = {}, None
    if not args.no_cpu:
        cpu, ref = cpu_baseline_leg(specs, masks, args)

    results = {}
    for v in variants:
        doms, batch, ms, ms2, tiles = run_variant(v, specs, masks, args.steps, args.warmup,
                                                  not args.no_tune,
                                                  parse_tiles(args.tiles) if args.tiles else None,
                                                  two_step=not args.single_step)
        mlups = sites * args.steps / (ms * 1e-3) / 1e6
        mflups = fluid_sites * args.steps / (ms * 1e-3) / 1e6
        bytes_alg = algorithmic_bytes(specs, masks, STORAGE_BYTES[v])
        gbs = bytes_alg * args.steps / (ms * 1e-3) / 1e9
        two = all(d.get_option(lb.OPT_TWO_STEP) == 1 for d in doms)
        spl = 2 if (two and args.steps % 4 == 0) else 1
        # average sweep launch: the extra steps of the 2K-step call over the
        # K-step one, per launch (the per-call density sums cancel)
        launch_ms = (ms2 - ms) / (args.steps / spl)
        entry = {"mlups": round(mlups, 1), "mflups": round(mflups, 1), "ms_per_step": round(ms / args.steps, 4),
                 "sweep_launch_ms": round(launch_ms, 4), "steps_per_launch": spl,
                 "sweep_GBps": round(spl * bytes_alg / (launch_ms * 1e-3) / 1e9, 1),
                 "hbm_frac": round(spl * bytes_alg / (launch_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                 "bytes_per_step": bytes_alg, "rounding": ROUNDING[v],
                 "two_step": two,
                 "tiles": tiles if isinstance(tiles, str) or tiles is None else {f"{'obstacles' if k[0] else 'open'}/class{k[1]}": f"{t[0]}x{t[1]}"
                                                       for k, t in tiles.items()}}
        results[v] = entry
        batch.close()
        for d in doms:
            d.close()
        del doms, batch
        torch.cuda.empty_cache()
        if ref:
            entry["l2_vs_oracle"] = accuracy_leg(v, specs, masks, ref)
        log(f"{v}: {json.dumps(entry)}")

    head = results[variants[0]]
    achieved = head["sweep_GBps"]
    # the workload's domains are periodic without particles, so with the
    # two-step option on (the default) every launch of the timed run is the
    # two-step sweep when the step count is a multiple of four
    spl = head["steps_per_launch"]
    copy_gbs = copy_bandwidth()
    log(f"device-to-device copy: {copy_gbs:.0f} GB/s")
    traffic = traffic_entry(spl)
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic,
                # bytes that really crossed HBM per launch (profiled) over the
                # launch duration: with two steps per launch the algorithmic
                # rate above is an effective one and exceeds this
                "measured_GBps": (None if traffic is None else
                                  round(traffic / (head["sweep_launch_ms"] * 1e-3) / 1e9, 1)),
                "launch_ms": head["sweep_launch_ms"],
                "kernel": (f"k_sweep2 (two steps per launch, {variants[0]} storage, batched)" if spl == 2
                           else f"k_sweep ({variants[0]} storage, batched)"),
                "steps_per_launch": spl,
                "algorithmic_bytes_per_launch": spl * head["bytes_per_step"],
                "copy_GBps": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4)}
    # the 16-bit two-step sweep is bound by vector issue as much as by memory:
    # the profile's VALU lane-instructions per site update and issue fraction
    prof = profile_entry(spl)
    if prof is not None and prof.get("valu"):
        roofline["valu_per_site_update"] = round(prof["valu"]["valu_per_site_update"], 1)
        roofline["valu_issue_frac"] = round(prof["valu"]["valu_issue_util"], 3)
    configs = replicas = offload = None
    if not args.no_configs:
        t0 = time.time()
        configs = other_configs()
        log(f"other workloads ({time.time() - t0:.0f}s): {json.dumps(configs)}")
        t0 = time.time()
        replicas = paper_replicas()
        log(f"paper benchmarks ({time.time() - t0:.0f}s): {json.dumps(replicas)}")
        t0 = time.time()
        offload = reporting_offload()
        log(f"reporting offload ({time.time() - t0:.0f}s): {json.dumps(offload)}")
    out = {
        "metric": METRIC, "value": head["mlups"], "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "precision-and-batching stress: 8192^2 periodic domain + 200 "
                               "uneven 64^2..2048^2 obstacle domains (20% solid), batched, "
                               f"{variants[0]}-delta storage",
                   "sites": sites, "domains": len(specs), "storage": variants[0],
                   "rounding": ROUNDING[variants[0]], "arithmetic": "f32"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "variants": results,
        "other_workloads": configs,
        "paper_benchmarks": replicas,
        "reporting_offload": offload,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
