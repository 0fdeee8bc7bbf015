"""Benchmark of the explicit 3-D diffusion step with periodic halo update on
one MI355X.

Workload (value): 512^3 FP64 local grid, 1x1x1 periodic topology, overlap 2,
lam = 1, dx = 1/(n-1), T0 = 1.7 + Gaussian bump, Ci lognormal(log 0.5, 0.2)
from seed 0, dt from maximum(Ci); every step is diffusion_step with
boundary-first split (16, 2, 2): the y and z boundary slabs and the halo
update of T2 (pack, exchange, unpack of the y and z planes) on the helper
stream, the inner region and x slabs on the caller stream, the x exchange
stored by the step kernels.  A step = one such call; K steps are timed after
W warm-up steps, with inputs already resident in HBM.

value = T_eff = (bytes of T read + Ci read + T2 written, each once per point)
/ time per step, in GB/s (decimal), the time per step being the median of 20
timings of K steps each (the paper's statistic); the first timed pass of K
steps is reported beside it (ms_per_step_single_pass).

Also reported on the same line:
  roofline      the inner-region step kernel: algorithmic bytes per launch
                over its average duration, timed live with HIP events on
                the stream it runs on during a second timed pass of the same
                K steps (so the events do not perturb `value`), against the
                8 TB/s HBM3E peak;
  ms_per_step_samples
                the 20 timings of K steps: median and its 95% interval;
  halo_overhead the split step's median over the median duration of the
                step kernel alone on every inner point (the unsplit step's
                kernel, without its halo update), minus 1; the unsplit
                step's own median is in variants.f64_unsplit;
  stream_ceiling_GBs
                the library's streaming probe (igg_stream_probe) on 1 GiB
                arrays for the read/write mixes of the step (2R1W), the
                adjoint (4R2W) and the fused flux pass (2R4W): the rate a
                plain stream reaches on this device;
  cpu_baseline  the CPU oracle on the host cores: 100 steps of the same
                512^3 workload (bounded to about 10-30 s), as T_eff, and
                one step on one core;
  variants      FP32 and FP16-storage steps at 512^3 (noisy-bump recipe,
                uniform Ci) with their error against the FP64 oracle (the
                GPU's FP64 result when the oracle is skipped), the
                unsplit FP64 step, the checkpointed adjoint at 256^3, the
                32^3 launch-bound step (eager and graph), and the 768^3
                staggered flux form in FP32 with its checkpointed adjoint.
"""
import argparse
import hashlib
import re
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "T_eff GB/s & % HBM peak per step, 512^3 FP64 vs FP32 fwd, and adjoint"
HBM_PEAK_GBS = 8000.0
SPLIT = (16, 2, 2)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=100)
    p.add_argument("--warmup", type=int, default=10)
    p.add_argument("--n", type=int, default=512, help="cube edge of the headline workload")
    p.add_argument("--no-variants", action="store_true", help="headline FP64 run only")
    p.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    p.add_argument("--samples", type=int, default=20,
                   help="extra timings of --steps steps for the median and its 95%% interval")
    p.add_argument("--profile", action="store_true",
                   help="headline loop only, for running under rocprofv3")
    p.add_argument("--profile-adjoint", type=int, default=0, metavar="N",
                   help="for rocprofv3 only: the calibration stream, then 6 unsplit FP64 adjoint steps at N^3")
    p.add_argument("--profile-flux", type=int, default=0, metavar="N",
                   help="for rocprofv3 only: the calibration stream, then 6 FP32 flux-form steps at N^3")
    p.add_argument("--profile-dtype", default="f64", choices=["f64", "f32", "f16", "f16rn"],
                   help="with --profile: element type of the profiled steps (the headline fields rounded once; "
                        "f16 with stochastic rounding, f16rn with round-to-nearest stores)")
    p.add_argument("--split", default="16,2,2",
                   help="boundary widths of the timed steps, or 'none' for the unsplit schedule")
    return p.parse_args()


def code_hash(sources):
    """Hash of C++ source texts with comments and layout dropped."""
    h = hashlib.sha256()
    for src in sources:
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def kernel_source_hash():
    """Hash of the code of the sources the inner step kernel is built from,
    so an edit of a comment keeps the counters taken on that kernel valid."""
    texts = []
    for f in ("step.hip", "device.hpp"):
        with open(os.path.join(ROOT, "paper_2211_15716_amd", "csrc", f)) as fh:
            texts.append(fh.read())
    return code_hash(texts)


def traffic_from_profiles(kernel_hash, key):
    """HBM bytes per launch measured by rocprofv3 PMC runs, if they were taken
    on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    e = rec.get(key)
    if not e or e.get("kernel_source_hash") != kernel_hash:
        return None
    return e.get("bytes_per_launch")


def time_steps(igg, torch, T, W, C, lam, dt, dx, dy, dz, steps, warmup, split, rnd_seed=None):
    """Do `warmup` untimed steps, then time exactly `steps` steps (the step
    time); then time the same number of steps again with the library's
    kernel timing events on the streams the kernels run on (HIP events,
    live, in this process), which give the inner-kernel and boundary
    durations without perturbing the first timing.  Returns (ms/step, final
    buffer of the first timed pass, inner-kernel ms/launch, inner
    points/launch, boundary-kernel ms per step, ms/step of the pass with the
    kernel events)."""
    a, b = T, W
    it = 0

    def one():
        nonlocal a, b, it
        rnd = igg.rounding("stochastic", rnd_seed, it) if rnd_seed is not None else None
        igg.diffusion_step(b, a, C, lam, dt, dx, dy, dz, split=split, rnd=rnd)
        a, b = b, a
        it += 1

    def timed():
        s0 = torch.cuda.Event(enable_timing=True)
        s1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s0.record()
        for _ in range(steps):
            one()
        s1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return max(wall * 1e3, s0.elapsed_time(s1)) / steps

    for _ in range(warmup):
        one()
    ms = timed()
    final = a
    if steps > 0:
        # the instrumented pass continues from the final state in fresh buffers
        a, b = a.clone(), b.clone()
    igg.timing_read()  # discard
    igg.timing_enable(True)  # the library makes its event pool here, before the pass
    ms_inst = timed()
    igg.timing_enable(False)
    k_ms, k_launches, k_points, b_ms = igg.timing_read()
    per_launch = k_ms / max(1, k_launches)
    return ms, final, per_launch, (k_points // max(1, k_launches)), b_ms / max(1, steps), ms_inst


def oracle_256_timings(oracle, synth, nthreads):
    """The oracle's forward and adjoint step on the 256^3 inverse-problem
    fields, on all threads and on one: median of 3 timings each, in ms."""
    import numpy as np
    w = synth.workload("c4_256_inverse", seed=0)
    T, C = w["T0"].copy(), w["Ci"].copy()
    oracle.halo(T)
    oracle.halo(C)
    d = (w["dx"], w["dy"], w["dz"])
    dt = oracle.time_step(*d, w["lam"], oracle.max_all(C))
    out, g = np.empty_like(T), np.zeros_like(T)

    def med(f):
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            f()
            ts.append(time.perf_counter() - t0)
        return round(sorted(ts)[1] * 1e3, 2)

    res = {"grid": [256, 256, 256]}
    for label, nth in (("all_cores", nthreads), ("1_core", 1)):
        oracle.set_num_threads(nth)
        res[f"forward_ms_{label}"] = med(lambda: oracle.step(T, C, w["lam"], dt, *d, out=out))
        res[f"adjoint_ms_{label}"] = med(lambda: oracle.adjoint_step(T, T, C, g, w["lam"], dt, *d, out=out))
    oracle.set_num_threads(nthreads)
    return res


def step_samples(igg, torch, T, C, lam, dt, dx, dy, dz, steps, split, n, rnd_seed=None):
    """n timings of `steps` steps each, continuing from T in fresh buffers
    (FP16 stores rounded stochastically when rnd_seed is given): median
    ms/step and the distribution-free 95% interval of the median (order
    statistics; for n = 20 the 6th and 15th values)."""
    if n < 1 or steps < 1:
        return None
    from math import comb
    a, b = T.clone(), T.clone()
    vals = []
    it = 0
    for _ in range(n):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(steps):
            rnd = igg.rounding("stochastic", rnd_seed, it) if rnd_seed is not None else None
            igg.diffusion_step(b, a, C, lam, dt, dx, dy, dz, split=split, rnd=rnd)
            a, b = b, a
            it += 1
        e1.record()
        torch.cuda.synchronize()
        vals.append(e0.elapsed_time(e1) / steps)
    vals.sort()
    med = vals[n // 2] if n % 2 else 0.5 * (vals[n // 2 - 1] + vals[n // 2])
    # largest k with P(Binomial(n, 1/2) < k) <= 2.5%: [x_(k), x_(n+1-k)] covers the median with >= 95%
    k, cdf = 0, 0.0
    while k < n // 2:
        p = comb(n, k) / 2.0 ** n
        if cdf + p > 0.025:
            break
        cdf += p
        k += 1
    lo, hi = (vals[k - 1], vals[n - k]) if k >= 1 else (vals[0], vals[-1])
    del a, b
    return {"n": n, "steps_each": steps, "median": round(med, 5), "ci95": [round(lo, 5), round(hi, 5)],
            "min": round(vals[0], 5), "max": round(vals[-1], 5)}


def kernel_samples(igg, torch, T, C, lam, dt, dx, dy, dz, steps, n):
    """n timings of `steps` unsplit steps with the library's kernel timing
    events: the median duration of the step kernel over every inner point
    (the step without its halo update), in ms."""
    if n < 1 or steps < 1:
        return None
    a, b = T.clone(), T.clone()
    vals = []
    igg.timing_read()
    igg.timing_enable(True)
    for _ in range(n):
        for _ in range(steps):
            igg.diffusion_step(b, a, C, lam, dt, dx, dy, dz, split=None)
            a, b = b, a
        k_ms, k_launches, _, _ = igg.timing_read()
        vals.append(k_ms / max(1, k_launches))
    igg.timing_enable(False)
    vals.sort()
    del a, b
    return vals[n // 2] if n % 2 else 0.5 * (vals[n // 2 - 1] + vals[n // 2])


def stream_ceilings(igg, torch, n_doubles=1 << 27, reps=10):
    """GB/s of the library's streaming probe for the step's, the adjoint's
    and the fused flux pass's read/write mixes (and a plain copy), on arrays
    of n_doubles doubles."""
    out = {}
    arrs = [torch.full((n_doubles,), 1.0 + q, dtype=torch.float64, device="cuda") for q in range(6)]
    for name, nr, nw in (("1R1W", 1, 1), ("2R1W", 2, 1), ("4R2W", 4, 2), ("2R4W", 2, 4)):
        src, dst = arrs[:nr], arrs[nr:nr + nw]
        for _ in range(2):
            igg.stream_probe(src, dst)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            igg.stream_probe(src, dst)
        e1.record()
        torch.cuda.synchronize()
        out[name] = round((nr + nw) * 8.0 * n_doubles * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
    del arrs
    torch.cuda.empty_cache()
    return out


def cpu_model():
    """The host CPU's model name (Linux), or the platform's processor string."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def calibration_stream(igg, torch):
    """A plain stream of known size ahead of the profiled kernels, the
    reference that scales the HBM byte counters of a profiling run: the
    streaming probe's 1R1W form on 2^27 doubles (1 GiB read, 1 GiB
    written)."""
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    igg.stream_probe([src], [dst])
    torch.cuda.synchronize()
    del src, dst


def profile_adjoint(igg, torch, synth, n):
    """The adjoint kernel alone, for HBM byte counters: the calibration
    stream, then 6 unsplit FP64 adjoint steps on n^3 fields (uniform random
    lam', T_n, Ci; gCi from 0)."""
    calibration_stream(igg, torch)
    igg.init_global_grid(n, n, n, dims=(1, 1, 1), periods=(1, 1, 1), overlaps=(2, 2, 2))
    lp, Tn, Ci = (torch.from_numpy(a).cuda() for a in synth.uniform_fields(n, n, n, seed=3, lo=0.5, hi=1.5, n=3))
    igg.update_halo(lp, Tn, Ci)
    ln, gCi = torch.zeros_like(lp), torch.zeros_like(lp)
    dx = 1.0 / (n - 1)
    dt = dx * dx / 1.5 / 6.1
    for _ in range(6):
        igg.diffusion_step_adjoint(ln, lp, Tn, Ci, gCi, 1.0, dt, dx, dx, dx, split=None)
        ln, lp = lp, ln
    torch.cuda.synchronize()
    igg.finalize_global_grid()
    print(json.dumps({"profile_adjoint": n, "points_per_launch": (n - 2) ** 3, "bytes_per_point": 48}), flush=True)


def profile_flux(igg, torch, synth, n):
    """The fused flux-form pass alone, for HBM byte counters: the calibration
    stream, then 6 unsplit FP32 flux-form steps on n^3 cells (the 768^3
    recipe at edge n)."""
    from paper_2211_15716_amd import diffusion
    calibration_stream(igg, torch)
    w = synth.workload("c5_768_flux", seed=0, n=n)
    igg.init_global_grid(n, n, n, dims=(1, 1, 1), periods=(1, 1, 1), overlaps=(2, 2, 2))
    T, C = diffusion.prepare_fields(w["T0"], w["Ci"], torch.float32)
    d = (w["dx"], w["dy"], w["dz"])
    dt = igg.diffusion_dt(C, w["lam"], *d)
    prob = diffusion.FluxProblem(w["lam"], dt, *d)
    diffusion.forward_with(prob, T, C, 6)
    torch.cuda.synchronize()
    igg.finalize_global_grid()
    print(json.dumps({"profile_flux": n, "cells_per_launch": (n - 2) ** 3, "bytes_per_cell_fused": 24}), flush=True)


def profile_step(igg, torch, synth, args):
    """For rocprofv3 runs: the calibration stream, then the headline loop
    alone (W warm-up and K timed steps of the 512^3 workload with its split,
    the fields rounded once to --profile-dtype; FP16 stores rounded
    stochastically as in the precision variant)."""
    calibration_stream(igg, torch)
    n = args.n
    w = synth.workload("c2_512_fp64", seed=0, n=n)
    d = (w["dx"], w["dy"], w["dz"])
    tdt = {"f64": torch.float64, "f32": torch.float32, "f16": torch.float16, "f16rn": torch.float16}[args.profile_dtype]
    igg.init_global_grid(n, n, n, dims=(1, 1, 1), periods=(1, 1, 1), overlaps=(2, 2, 2))
    T = torch.from_numpy(w["T0"]).cuda().to(tdt).contiguous()
    C = torch.from_numpy(w["Ci"]).cuda().to(tdt).contiguous()
    del w
    igg.update_halo(T, C)
    dt = igg.diffusion_dt(C, 1.0, *d)
    split = None if args.split == "none" else tuple(int(v) for v in args.split.split(","))
    seed = 1234 if args.profile_dtype == "f16" else None
    ms, _, k_ms, k_pts, _, _ = time_steps(igg, torch, T, T.clone(), C, 1.0, dt, *d, args.steps, args.warmup, split,
                                          rnd_seed=seed)
    igg.finalize_global_grid()
    print(json.dumps({"profile": args.profile_dtype, "grid": [n, n, n], "split": args.split, "ms_per_step": ms,
                      "kernel_ms": k_ms, "points_per_launch": k_pts, "bytes_per_point": 3 * T.element_size(),
                      "kernel_source_hash": kernel_source_hash()}), flush=True)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this library has no multi-GPU path "
              "(the halo exchange is a self-exchange on a 1x1x1 periodic topology); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2211_15716_amd import igg, synth

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    if args.profile_adjoint:
        profile_adjoint(igg, torch, synth, args.profile_adjoint)
        return
    if args.profile_flux:
        profile_flux(igg, torch, synth, args.profile_flux)
        return
    if args.profile_dtype != "f64" and not args.profile:
        raise SystemExit("--profile-dtype is for --profile runs only")
    torch.cuda.set_device(0)
    n = args.n
    K, Wm = args.steps, args.warmup

    if args.profile:
        profile_step(igg, torch, synth, args)
        return

    # ---------------------------------------------------------------- headline FP64
    log(f"generating {n}^3 FP64 inputs (bump + lognormal Ci, seed 0)")
    w = synth.workload("c2_512_fp64", seed=0, n=n)
    lam, dx, dy, dz = w["lam"], w["dx"], w["dy"], w["dz"]
    pts = n ** 3
    igg.init_global_grid(n, n, n, dims=(1, 1, 1), periods=(1, 1, 1), overlaps=(2, 2, 2))
    T = torch.from_numpy(w["T0"]).cuda()
    C = torch.from_numpy(w["Ci"]).cuda()
    igg.update_halo(T, C)
    T0_dev = T.clone()
    dt = igg.diffusion_dt(C, lam, dx, dy, dz)
    Wb = T.clone()  # the second buffer starts as a copy (Fig. 1)
    log(f"timing {K} FP64 steps after {Wm} warm-up steps, split {args.split}")
    split = None if args.split == "none" else tuple(int(v) for v in args.split.split(","))
    ms1, out64, k_ms, k_pts, b_ms, ms_inst = time_steps(igg, torch, T, Wb, C, lam, dt, dx, dy, dz, K, Wm, split)
    samples = step_samples(igg, torch, out64, C, lam, dt, dx, dy, dz, K, split, 0 if args.profile else args.samples)
    # the step time is the median of the samples (the first pass alone when
    # there are none)
    ms = samples["median"] if samples else ms1
    teff = 24.0 * pts / (ms * 1e-3) / 1e9
    k_bytes = 24.0 * k_pts
    k_gbs = k_bytes / (k_ms * 1e-3) / 1e9
    khash = kernel_source_hash()
    traffic = traffic_from_profiles(khash, "step_f64_512")
    log(f"FP64: {ms:.4f} ms/step (median; first pass {ms1:.4f}), T_eff {teff:.1f} GB/s; "
        f"step kernel {k_ms:.4f} ms, {k_gbs:.1f} GB/s")

    result = {
        "metric": METRIC, "value": round(teff, 2), "unit": "GB/s", "n_gpus": 1, "steps": K,
        "warmup": Wm, "ms_per_step": round(ms, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"explicit 3-D diffusion step + periodic halo update, {n}^3 FP64, "
                               f"1x1x1 periodic topology, overlap 2, split {args.split}, bump T0, "
                               f"lognormal Ci (seed 0)",
                   "grid": [n, n, n], "nt_timed": K, "split": None if split is None else list(split), "dt": dt,
                   "bytes_per_point": 24, "parallelism": "1 GPU"},
        "hbm_frac": round(teff / HBM_PEAK_GBS, 4),
        "roofline": {"bound": "hbm",
                     "kernel": "k_step_zmarch<double> (inner region; with the default one-launch schedule also "
                               "the y/z boundary slabs, by its first work-groups)",
                     "achieved": round(k_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(k_gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "bytes_per_launch": k_bytes, "points_per_launch": k_pts,
                     "ms_per_launch": round(k_ms, 5), "kernel_source_hash": khash},
        "halo_overhead": None,
        "ms_per_step_single_pass": round(ms1, 5),
        "ms_per_step_samples": samples,
        "boundary_ms_per_step": round(b_ms, 5),
        "ms_per_step_with_kernel_events": round(ms_inst, 5),
    }


    # ---------------------------------------------------------------- streaming ceiling of the mixes
    result["stream_ceiling_GBs"] = stream_ceilings(igg, torch)
    ceil = result["stream_ceiling_GBs"]["2R1W"]
    result["roofline"]["frac_of_stream_ceiling"] = round(k_gbs / ceil, 4)
    log(f"streaming probe (GB/s): {result['stream_ceiling_GBs']}")

    # ---------------------------------------------------------------- unsplit FP64 for comparison
    nsu = max(1, args.samples)
    u_samples = step_samples(igg, torch, T0_dev, C, lam, dt, dx, dy, dz, K, None, nsu)
    ku_ms = kernel_samples(igg, torch, T0_dev, C, lam, dt, dx, dy, dz, K, nsu)
    ms_u = u_samples["median"]
    result["variants"] = {"f64_unsplit": {"ms_per_step": ms_u,
                                          "T_eff_GBs": round(24.0 * pts / (ms_u * 1e-3) / 1e9, 1),
                                          "kernel_ms": round(ku_ms, 5), "ms_per_step_samples": u_samples}}
    # the halo update's step-time overhead: the split step against the step
    # kernel over all inner points alone (the same computation, no update),
    # both medians of this run
    if split is not None:
        result["halo_overhead"] = round(ms / ku_ms - 1.0, 4)
        result["split_vs_unsplit_step"] = round(ms / ms_u, 4)
    log(f"unsplit: step {ms_u:.4f} ms, kernel alone {ku_ms:.4f} ms (medians); "
        f"split {ms:.4f} ms: halo overhead {result['halo_overhead']}")

    # ---------------------------------------------------------------- CPU oracle baseline
    gpu64 = None
    if not args.no_cpu:
        import oracle
        oracle_nt = K if K <= 100 else 100
        T0h, Cih = w["T0"].copy(), w["Ci"].copy()
        oracle.halo(T0h)
        oracle.halo(Cih)
        # the GPU result after exactly oracle_nt steps, for a full-field error
        T = T0_dev.clone()
        ms_chk, gout, _, _, _, _ = time_steps(igg, torch, T, Wb, C, lam, dt, dx, dy, dz, oracle_nt, 0, SPLIT)
        gpu64 = gout.cpu().numpy()
        log(f"oracle: up to {oracle_nt} steps of the {n}^3 FP64 workload on the host")
        cur, nxt = T0h, np.empty_like(T0h)
        nxt[...] = cur
        # the oracle steps for at least 10 s (at most 30 s) so the timing is a
        # stable sample; after oracle_nt steps its state is compared with the
        # GPU's (that comparison is not timed)
        t0 = time.perf_counter()
        paused = 0.0
        done = 0
        err = None
        while True:
            oracle.step(cur, Cih, lam, dt, dx, dy, dz, out=nxt)
            oracle.halo(nxt)
            cur, nxt = nxt, cur
            done += 1
            if done == oracle_nt:
                tp = time.perf_counter()
                err = oracle.rel_max_err(gpu64, cur)
                paused += time.perf_counter() - tp
            el = time.perf_counter() - t0 - paused
            if (done >= oracle_nt and el >= 10.0) or el > 30.0:
                break
        cpu_teff = 24.0 * pts * done / el / 1e9
        result["cpu_baseline"] = {"value": round(cpu_teff, 2), "unit": "GB/s", "cores": oracle.num_threads(),
                                  "cpu_model": cpu_model(), "kind": "oracle",
                                  "sample": f"{done} steps of the {n}^3 FP64 workload (plain C loops, "
                                            f"OpenMP over z), {el:.1f} s"}
        if err is not None:
            result["f64_err_vs_oracle"] = err
            log(f"FP64 GPU vs oracle after {oracle_nt} steps: {err:.3e}")
        # one step on one core, for the per-core figure
        nthreads = oracle.num_threads()
        oracle.set_num_threads(1)
        t1 = time.perf_counter()
        oracle.step(cur, Cih, lam, dt, dx, dy, dz, out=nxt)
        oracle.halo(nxt)
        one_core = time.perf_counter() - t1
        oracle.set_num_threads(nthreads)
        result["cpu_baseline"]["ms_per_step"] = round(el * 1e3 / done, 2)
        result["cpu_baseline"]["ms_per_step_1_core"] = round(one_core * 1e3, 1)
        log(f"oracle: {el * 1e3 / done:.1f} ms/step on {nthreads} threads, {one_core * 1e3:.1f} ms on one")
        del T0h, Cih, cur, nxt
        result["cpu_baseline"]["c4_256"] = oracle_256_timings(oracle, synth, nthreads)

    if args.no_variants:
        print(json.dumps(result), flush=True)
        igg.finalize_global_grid()
        return

    # ---------------------------------------------------------------- FP32 / FP16 variants
    log(f"generating {n}^3 noisy-bump inputs (uniform Ci, seed 0) for the precision forms")
    w3 = synth.workload("c3_512", seed=0, n=n)
    T0_64 = torch.from_numpy(w3["T0"]).cuda()
    C_64 = torch.from_numpy(w3["Ci"]).cuda()
    igg.update_halo(T0_64, C_64)
    dt3 = igg.diffusion_dt(C_64, lam, dx, dy, dz)
    nt3 = 100
    # the reference of the error: the FP64 oracle after nt3 steps (the GPU's
    # own FP64 run when the oracle leg is skipped)
    ref_np, ref_kind = None, "gpu_f64"
    if not args.no_cpu:
        import oracle
        T0h, Cih = w3["T0"].copy(), w3["Ci"].copy()
        oracle.halo(T0h)
        oracle.halo(Cih)
        if oracle.time_step(dx, dy, dz, lam, oracle.max_all(Cih)) != dt3:
            raise RuntimeError("GPU and oracle dt differ")
        log(f"oracle: {nt3} steps of the precision-form workload (error reference)")
        ref_np, ref_kind = oracle.run(T0h, Cih, nt3, lam, dt3, dx, dy, dz), "oracle"
        del T0h, Cih

    def run_nt3(Tv, Cv, seed, offset=0.0):
        a, b = Tv.clone(), torch.empty_like(Tv)
        for it in range(nt3):
            rnd = igg.rounding("stochastic", seed, it) if seed is not None else None
            igg.diffusion_step(b, a, Cv, lam, dt3, dx, dy, dz, split=SPLIT, rnd=rnd)
            a, b = b, a
        return a.to(torch.float64) + offset

    def rel_err(final):
        if ref_np is not None:
            got = final.cpu().numpy()
            i = (slice(1, -1),) * 3
            return float(np.max(np.abs(got[i] - ref_np[i])) / np.max(np.abs(ref_np[i])))
        d = (final - gpu_ref)[1:-1, 1:-1, 1:-1].abs().max().item()
        return d / gpu_ref[1:-1, 1:-1, 1:-1].abs().max().item()

    gpu_ref = None
    for name, tdt in (("f64", torch.float64), ("f32", torch.float32), ("f16", torch.float16)):
        Tv = T0_64.to(tdt).contiguous()
        Cv = C_64.to(tdt).contiguous()
        Wv = torch.empty_like(Tv)
        seed = 1234 if name == "f16" else None
        final = run_nt3(Tv, Cv, seed)
        if name == "f64" and ref_np is None:
            gpu_ref = final
        err = rel_err(final)
        ms1v, _, kv_ms, kv_pts, _, _ = time_steps(igg, torch, Tv.clone(), Wv, Cv, lam, dt3, dx, dy, dz, K, Wm,
                                                  SPLIT, rnd_seed=seed)
        sv = step_samples(igg, torch, Tv, Cv, lam, dt3, dx, dy, dz, K, SPLIT, args.samples, rnd_seed=seed)
        msv = sv["median"] if sv else ms1v
        s = Tv.element_size()
        entry = {"ms_per_step": round(msv, 5), "ms_per_step_single_pass": round(ms1v, 5),
                 "T_eff_GBs": round(3 * s * pts / (msv * 1e-3) / 1e9, 1),
                 "hbm_frac": round(3 * s * pts / (msv * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                 "kernel_GBs": round(3 * s * kv_pts / (kv_ms * 1e-3) / 1e9, 1),
                 "err": err, "err_reference": ref_kind, "nt_err": nt3}
        if name == "f16":
            entry["rounding"] = "stochastic"
        result["variants"][name] = entry
        log(f"{name}: {msv:.4f} ms/step, err vs {ref_kind} {err:.3e}")
        del Tv, Cv, Wv, final
    f32 = result["variants"]["f32"]
    result["variants"]["f32_speedup_vs_f64"] = round(result["variants"]["f64"]["ms_per_step"] / f32["ms_per_step"], 3)
    # FP16 with round-to-nearest stores, for comparison of the error
    Cv = C_64.to(torch.float16).contiguous()
    result["variants"]["f16"]["err_round_nearest"] = rel_err(run_nt3(T0_64.to(torch.float16).contiguous(), Cv,
                                                                     None))
    # FP16 storage of T - 1.7 with stochastic rounding: the step is linear and
    # a constant field is a fixed point, so stepping T - c gives the same
    # scheme; the smaller stored values keep finer absolute resolution
    off = 1.7
    result["variants"]["f16"]["err_offset_1.7"] = rel_err(run_nt3((T0_64 - off).to(torch.float16).contiguous(), Cv,
                                                                  1234, off))
    del Cv, T0_64, C_64, gpu_ref, ref_np
    torch.cuda.empty_cache()

    igg.finalize_global_grid()

    # ---------------------------------------------------------------- checkpointed adjoint
    result["variants"]["adjoint_256"] = adjoint_variant(igg, torch, synth)
    # ---------------------------------------------------------------- small grid: eager vs graph
    result["variants"]["c1_32_launch_bound"] = small_grid_variant(igg, torch, synth)
    # ---------------------------------------------------------------- staggered flux form
    result["variants"]["flux_768_fp32"] = flux_variant(igg, torch, synth, K)

    print(json.dumps(result), flush=True)


def adjoint_variant(igg, torch, synth):
    """Loss and gradient of the 256^3 FP64 inverse problem: nt = 200 steps,
    T_obs from Ci_true (sine), guess Ci = 0.5, snapshots every 16 steps.
    Algorithmic bytes: 24 per point per forward step (forward sweep and
    recomputation) and 48 per point per adjoint step (lam', Ci, T_n read,
    gCi read and written, lam written)."""
    from paper_2211_15716_amd import diffusion
    w = synth.workload("c4_256_inverse", seed=0)
    n = w["nx"]
    nt = w["nt"]
    pts = n ** 3
    igg.init_global_grid(n, n, n, dims=(1, 1, 1), periods=(1, 1, 1), overlaps=(2, 2, 2))
    T, Ctrue = diffusion.prepare_fields(w["T0"], w["Ci"])
    dt = igg.diffusion_dt(Ctrue, w["lam"], w["dx"], w["dy"], w["dz"])
    prob = diffusion.Problem(w["lam"], dt, w["dx"], w["dy"], w["dz"], split=SPLIT)
    O = diffusion.forward(T.clone(), Ctrue, nt, prob.lam, dt, prob.dx, prob.dy, prob.dz, split=SPLIT)
    C = torch.full_like(T, 0.5)
    sched = ("periodic", 16)
    diffusion.loss_and_grad(T, C, O, prob, nt, sched)  # warm-up
    torch.cuda.synchronize()
    igg.timing_enable(True)
    t0 = time.perf_counter()
    L, gT, gC, sw = diffusion.loss_and_grad(T, C, O, prob, nt, sched)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    igg.timing_enable(False)
    k_ms, k_launches, k_pts, b_ms = igg.timing_read()
    nbytes = (24.0 * sw.advances + 48.0 * sw.adjoints) * pts
    # the same gradient with events between the sweeps: the reverse sweep's
    # own time (adjoint steps plus the recomputation inside each segment)
    sw2 = diffusion.Sweep(prob, C, T, diffusion.checkpoint_ops(*sched[:1], nt, *sched[1:]))
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    torch.cuda.synchronize()
    ev[0].record()
    Tnt = sw2.forward(nt)
    ev[1].record()
    fwd_adv = sw2.advances
    lam_nt = diffusion._inner_only(Tnt - O)
    igg.update_halo(lam_nt)
    sw2.reverse(lam_nt)
    ev[2].record()
    torch.cuda.synchronize()
    rev_ms = ev[1].elapsed_time(ev[2])
    recompute = sw2.advances - fwd_adv
    rev_bytes = (48.0 * sw2.adjoints + 24.0 * recompute) * pts
    out = {"grid": [n, n, n], "nt": nt, "schedule": "periodic every 16", "ms_total": round(el * 1e3, 3),
           "forward_steps": sw.advances, "adjoint_steps": sw.adjoints, "peak_snapshots": sw.peak,
           "T_eff_GBs": round(nbytes / el / 1e9, 1), "hbm_frac": round(nbytes / el / 1e9 / HBM_PEAK_GBS, 4),
           "forward_sweep_ms": round(ev[0].elapsed_time(ev[1]), 3),
           "ms_per_reverse_step": round(rev_ms / nt, 4),
           "reverse_recompute_steps": recompute,
           "reverse_T_eff_GBs": round(rev_bytes / (rev_ms * 1e-3) / 1e9, 1),
           "reverse_hbm_frac": round(rev_bytes / (rev_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "loss": L}
    rev_ms = rev_ms / nt
    log(f"adjoint 256^3: {el*1e3:.1f} ms, T_eff {out['T_eff_GBs']} GB/s, reverse step {rev_ms:.4f} ms")
    del T, Ctrue, O, C, gT, gC, sw, sw2, Tnt, lam_nt
    torch.cuda.empty_cache()
    igg.finalize_global_grid()
    return out


def flux_variant(igg, torch, synth, K):
    """768^3 staggered flux form in FP32 (cells 768^3, faces 769 x 768^2 per
    component): K timed steps (the fused face-and-cell pass, halo update of
    T2, qx, qy, qz); 100 steps in FP32 and FP64 for the error; the
    checkpointed adjoint (sqrt(nt) snapshots) of 0.5*||T_nt - T0||^2 over
    nt = 100 steps in FP32 and FP64, and the gradients' difference.
    Algorithmic bytes of the method as two passes: 10*s per cell per step
    (flux: T read, three faces written; update: T, Ci and three faces read,
    T2 written); the fused pass needs only 6*s (the faces are not read
    back), reported beside it."""
    from paper_2211_15716_amd import diffusion
    w = synth.workload("c5_768_flux", seed=0)
    n = w["nx"]
    d = (w["dx"], w["dy"], w["dz"])
    lam = w["lam"]
    nt = w["nt"]
    pts = float(n) ** 3
    igg.init_global_grid(n, n, n, dims=(1, 1, 1), periods=(1, 1, 1), overlaps=(2, 2, 2))
    T64, C64 = diffusion.prepare_fields(w["T0"], w["Ci"])
    del w
    dt = igg.diffusion_dt(C64, lam, *d)
    out = {"grid": [n, n, n], "nt": nt, "bytes_per_cell": 40}
    finals = {}
    for name, tdt in (("f32", torch.float32), ("f64", torch.float64)):
        T = T64.to(tdt).contiguous()
        C = C64.to(tdt).contiguous()
        prob = diffusion.FluxProblem(lam, dt, *d)
        a, b = T.clone(), T.clone()
        for _ in range(nt):
            prob.step(b, a, C)
            a, b = b, a
        finals[name] = a.to(torch.float64)
        if name == "f32":
            for _ in range(3):
                prob.step(b, a, C)
                a, b = b, a
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(K):
                prob.step(b, a, C)
                a, b = b, a
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / K
            # T_eff by the two-pass count (40 B per cell), and the rate of the
            # least traffic the fused pass needs (T, Ci read; T2, qx, qy, qz
            # written: 24 B per cell), which is what HBM actually has to carry
            out.update({"ms_per_step": round(ms, 4), "T_eff_GBs": round(40.0 * pts / (ms * 1e-3) / 1e9, 1),
                        "hbm_frac": round(40.0 * pts / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                        "fused_min_bytes_per_cell": 24,
                        "fused_min_traffic_GBs": round(24.0 * pts / (ms * 1e-3) / 1e9, 1),
                        "fused_min_traffic_frac": round(24.0 * pts / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)})
        del a, b
        # checkpointed adjoint, sqrt(nt) snapshots
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L, gT, gC, sw = diffusion.loss_and_grad(T, C, T, prob, nt, ("sqrt",))
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        finals[name + "_grad"] = (gT.to(torch.float64), gC.to(torch.float64))
        out[f"adjoint_{name}"] = {"ms_total": round(el * 1e3, 1), "forward_steps": sw.advances,
                                  "adjoint_steps": sw.adjoints, "peak_snapshots": sw.peak, "loss": L}
        del T, C, gT, gC, sw, prob
        torch.cuda.empty_cache()
    ref = finals["f64"][1:-1, 1:-1, 1:-1]
    out["err_f32_vs_f64"] = (finals["f32"][1:-1, 1:-1, 1:-1] - ref).abs().max().item() / ref.abs().max().item()
    for q, nm in ((0, "dT0"), (1, "dCi")):
        g64 = finals["f64_grad"][q][1:-1, 1:-1, 1:-1]
        g32 = finals["f32_grad"][q][1:-1, 1:-1, 1:-1]
        out[f"grad_{nm}_err_f32_vs_f64"] = (g32 - g64).abs().max().item() / g64.abs().max().item()
    del finals, ref, T64, C64
    torch.cuda.empty_cache()
    igg.finalize_global_grid()
    log(f"flux form 768^3 FP32: {out.get('ms_per_step')} ms/step, err vs FP64 {out['err_f32_vs_f64']:.2e}")
    return out


def small_grid_variant(igg, torch, synth):
    """32^3 FP64 (the parity workload): launch-bound, so eager steps are
    compared with replays of a captured HIP graph of the same steps."""
    from paper_2211_15716_amd import diffusion
    w = synth.workload("c1_32_fp64", seed=0)
    n = w["nx"]
    igg.init_global_grid(n, n, n, dims=(1, 1, 1), periods=(1, 1, 1), overlaps=(2, 2, 2))
    T, C = diffusion.prepare_fields(w["T0"], w["Ci"])
    d = (w["dx"], w["dy"], w["dz"])
    dt = igg.diffusion_dt(C, w["lam"], *d)
    T2 = T.clone()
    nsteps = 200
    diffusion.forward(T.clone(), C, 10, w["lam"], dt, *d, split=SPLIT)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    diffusion.forward(T.clone(), C, nsteps, w["lam"], dt, *d, split=SPLIT)
    torch.cuda.synchronize()
    eager = (time.perf_counter() - t0) * 1e3 / nsteps
    g = diffusion.StepGraph(T, T2, C, w["lam"], dt, *d, split=SPLIT, pairs=10)
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(nsteps // g.steps):
        g.replay()
    torch.cuda.synchronize()
    graph = (time.perf_counter() - t0) * 1e3 / nsteps
    # the library's own graph (diffusion_run): captured on the first call
    Tn, Tn2 = T.clone(), T.clone()
    igg.diffusion_run(Tn, Tn2, C, w["lam"], dt, *d, nsteps, split=SPLIT, graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    igg.diffusion_run(Tn, Tn2, C, w["lam"], dt, *d, nsteps, split=SPLIT, graph=True)
    torch.cuda.synchronize()
    native = (time.perf_counter() - t0) * 1e3 / nsteps
    igg.finalize_global_grid()
    log(f"32^3: eager {eager*1e3:.1f} us/step, graph {graph*1e3:.1f} us/step, library graph {native*1e3:.1f}")
    return {"grid": [n, n, n], "split": list(SPLIT), "eager_us_per_step": round(eager * 1e3, 2),
            "graph_us_per_step": round(graph * 1e3, 2), "steps_per_s_graph": round(1e3 / graph, 1),
            "library_graph_us_per_step": round(native * 1e3, 2)}


if __name__ == "__main__":
    main()
