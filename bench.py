#!/usr/bin/env python3
"""Benchmark: SHT+ISHT forward and backward fields/s at 721x1440, lmax 720.

One step = one pass of the whole path over the batch: SHT -> ISHT (forward)
then ISHT^T -> SHT^T (backward), i.e. four transforms of 72 fields on the
equiangular 721 x 1440 grid (both poles, Clenshaw-Curtis weights),
lmax = mmax = 720.  Inputs are resident in HBM before the timed region.

Prints ONE JSON line.  Besides the driver's contract fields it carries:
  roofline       -- the dominant kernel (Legendre contraction): FP32 against
                    the matrix-core peak with its algorithmic flops, the bf16
                    forms against HBM with their algorithmic bytes (folded
                    table in storage form + dense spectrum), per launch, over
                    its average launch time from HIP events recorded on the
                    launch stream during the timed region; step_frac is the
                    whole step against four such launches at that bound;
  cpu_baseline   -- the FP64 NumPy oracle doing the same four transforms on
                    the host (rank 0, N = 1): median of three passes after a
                    warm-up, the oracle's own Legendre recurrence timed apart;
  err_vs_fp64    -- relative L2 of each of the four GPU stages against the
                    oracle applied to that stage's own input;
  step_ms        -- p10 / p50 / p90 of the per-step HIP-event times;
  graph_replay_ms-- the same four transforms captured as one HIP graph.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SHT+ISHT fwd+bwd fields/sec at 721×1440 lmax720; % roofline; err vs FP64"
PEAKS_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "bf16x2": 2500.0, "bf16x3": 2500.0}
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16", "bf16x2", "bf16x3"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy a 256 MiB device buffer three times (reference kernel for HBM counters)")
    ap.add_argument("--cpu-fields", type=int, default=72,
                    help="fields in the oracle's timed sample (of the 72)")
    ap.add_argument("--workload", default="sht721", choices=["sht721", "batched", "sfno_block", "scores", "noise"],
                    help="sht721: the headline single-grid step; batched: uneven grids in one plan, "
                         "graph-replayed, with p50/p99 replay latency")
    ap.add_argument("--tune-cache", default=None, help="autotuner cache file (batched workload)")
    ap.add_argument("--schedule", default=None,
                    help="chunk,policy,ncb[,staged]: an explicit work schedule for the Legendre kernels "
                         "(results unchanged)")
    ap.add_argument("--tune", action="store_true", help="run the schedule autotuner before timing (sht721)")
    ap.add_argument("--block-batch", type=int, default=4, help="sfno_block: batch (ensemble members)")
    ap.add_argument("--profile-run", action="store_true",
                    help="sht721: skip the graph replay and the peak microbenchmarks after the timed region, so "
                         "that a profiler sees only the plan build, the warm-up and the timed steps")
    ap.add_argument("--block-channels", type=int, default=256, help="sfno_block: channels (677 in the model)")
    ap.add_argument("--replays", type=int, default=1000, help="batched: timed graph replays (p50 / p99 over them)")
    ap.add_argument("--replay-warmup", type=int, default=50, help="batched: untimed replays first")
    return ap.parse_args()


def legendre_flops(nlat, lmax, mmax, fields):
    """Multiply-adds x 2 of one folded Legendre contraction launch: every
    (l, m) pair with m <= l meets the nk = (nlat+1)/2 northern rings once per
    real column (2 per field)."""
    nk = (nlat + 1) // 2
    pairs = sum(lmax - m for m in range(mmax))
    return 2.0 * pairs * nk * 2 * fields


# matrix-core products per multiply-add of each form (split forms: the
# products a_i b_j the kernels form)
PRODUCTS = {"fp32": 1, "bf16": 1, "bf16x2": 5, "bf16x3": 6}
TABLE_BYTES = {"fp32": 4, "bf16": 2, "bf16x2": 4, "bf16x3": 6}


def legendre_bytes(nlat, lmax, mmax, fields, precision):
    """Algorithmic HBM bytes of one folded Legendre contraction launch: the
    table of every (l, m) pair at the nk northern rings once, in its storage
    form, plus the dense complex64 spectrum [fields][lmax][mmax] once.  The
    DFT intermediate is an implementation cost and is not counted."""
    nk = (nlat + 1) // 2
    pairs = sum(lmax - m for m in range(mmax))
    return pairs * nk * TABLE_BYTES[precision] + fields * lmax * mmax * 8


def profiled_traffic(kind, precision, extra=None):
    """HBM bytes per launch of the dominant kernel (plus, with extra, of the
    transpose or staging kernel charged to it) from the committed rocprofv3
    summary (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy of known
    size), or None when there is no summary for this precision or a kernel
    source has changed since the counters were taken."""
    import glob
    import hashlib

    def sha(name):
        with open(os.path.join(ROOT, "paper_2507_12144_amd", "csrc", name), "rb") as fh:
            return hashlib.sha256(fh.read()).hexdigest()[:16]

    want = {"legendre" if precision == "fp32" else "legendre_bf16":
            sha("legendre.h" if precision == "fp32" else "legendre_bf16.h")}
    if extra:
        want["transpose"] = sha("transpose.hip")
    prefixes = ["analysis" if kind == "legendre_analysis" else "synthesis"] + ([extra] if extra else [])
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(path) as fh:
            for line in fh:
                if not line.startswith("traffic_json: "):
                    continue
                rec = json.loads(line[len("traffic_json: "):])
                if rec.get("precision") != precision or any(rec["source_sha256_16"].get(k) != v
                                                            for k, v in want.items()):
                    continue
                got = [v for pre in prefixes for name, v in rec["hbm_bytes_per_launch"].items()
                       if name.startswith(pre)]
                if len(got) == len(prefixes):
                    return {"hbm_bytes_per_launch": sum(got), "source": os.path.relpath(path, ROOT)}
    return None


def calibrate_copy():
    """Plain device-to-device copies of known size: the reference that scales
    rocprofv3's FETCH_SIZE / WRITE_SIZE readings to bytes."""
    import torch
    torch.cuda.set_device(0)
    n = 1 << 26  # 256 MiB of float32
    a = torch.ones(n, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_bytes": 4 * n, "copies": 3}), flush=True)


# 16 ensemble members over three equiangular grids (poles included,
# Clenshaw-Curtis weights), 72 channels each
BATCHED_SEGMENTS = [  # nlat, nlon, lmax, members
    (181, 360, 180, 5),
    (361, 720, 360, 5),
    (721, 1440, 720, 6),
]


def batched_bench(args):
    """One plan over the three grids; the fwd+bwd chain SHT -> ISHT -> ISHT^T
    -> SHT^T over all 16 x 72 fields captured as one HIP graph after the
    schedule autotuner ran; --replays timed replays (default 1000) after
    --replay-warmup untimed ones (default 50), each timed with HIP events."""
    import numpy as np
    import torch
    import paper_2507_12144_amd as P
    torch.cuda.set_device(0)
    C = 72
    descs = [dict(nlat=a, nlon=b, lmax=L, mmax=L, grid="equiangular", batch=B, channels=C)
             for a, b, L, B in BATCHED_SEGMENTS]
    fields = sum(B for *_, B in BATCHED_SEGMENTS) * C
    t0 = time.perf_counter()
    plan = P.Plan(descs, precision=args.precision)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    choice, tune_ms = plan.tune(args.tune_cache)
    tune_s = time.perf_counter() - t0
    gen = torch.Generator(device="cuda")
    gen.manual_seed(0)
    u = torch.randn(plan.grid_shape(), device="cuda", generator=gen)
    y = torch.empty(plan.spec_shape(), dtype=torch.complex64, device="cuda")
    x = torch.empty(plan.grid_shape(), dtype=torch.float32, device="cuda")
    gy, gx = torch.empty_like(y), torch.empty_like(x)
    graph = plan.graph([("sht", u, y), ("isht", y, x), ("isht_T", x, gy), ("sht_T", gy, gx)])
    stream = torch.cuda.current_stream()
    n, warm = args.replays, args.replay_warmup
    for _ in range(warm):
        graph.launch()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    t0 = time.perf_counter()
    for a, b in evs:
        a.record(stream)
        graph.launch()
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = np.array([a.elapsed_time(b) for a, b in evs])
    out = {
        "metric": "batched uneven-grid SHT+ISHT fwd+bwd fields/sec (one plan, graph replay); p50/p99 replay latency",
        "value": round(fields * n / wall, 1), "unit": "fields/s", "n_gpus": 1, "steps": n,
        "warmup": warm, "ms_per_step": round(wall * 1e3 / n, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32" if args.precision == "fp32" else args.precision,
        "data": "synthetic",
        "config": {"workload": "16 ensemble members x 72 channels over equiangular 181x360 (L180), 361x720 "
                               "(L360) and 721x1440 (L720) grids in one plan; SHT->ISHT->ISHT^T->SHT^T "
                               "captured as one HIP graph",
                   "segments": [dict(nlat=a, nlon=b, lmax=L, members=B, channels=C) for a, b, L, B in
                                BATCHED_SEGMENTS],
                   "fields": fields, "precision": args.precision},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4), "p99": round(float(np.percentile(lat, 99)), 4),
                       "min": round(float(lat.min()), 4), "max": round(float(lat.max()), 4)},
        "tuner": {"chosen": choice, "best_pass_ms": round(tune_ms, 3), "seconds": round(tune_s, 2)},
        "plan_build_s": round(plan_s, 3),
    }
    print(json.dumps(out), flush=True)
    graph.close()
    plan.close()


def sfno_block_bench(args):
    """The spectral-convolution block y = ISHT(mix_W(SHT(x))) on a Gauss
    360 x 720 grid, lmax = mmax = 360, 4 x 256 channels, forward and backward
    with the weight gradient: SHT, mix, ISHT, then ISHT^T, mix^T, dW, SHT^T
    (FP32).  Per-kernel times from HIP events on the launch stream; the
    roofline of the channel-mix kernels (mix, mix^T and dW: per launch
    8 C^2 sum_l B min(l + 1, mmax) flops) is against the FP32 matrix-core
    peak (the kernels run on v_mfma_f32_16x16x4_f32)."""
    import numpy as np
    import torch
    import paper_2507_12144_amd as P
    torch.cuda.set_device(0)
    nlat, nlon, L, B, C = 360, 720, 360, args.block_batch, args.block_channels
    plan = P.Plan(dict(nlat=nlat, nlon=nlon, lmax=L, mmax=L, grid="gauss", batch=B, channels=C))
    if args.schedule:
        plan.set_schedule(*[int(v) for v in args.schedule.split(",")])
    gen = torch.Generator(device="cuda")
    gen.manual_seed(0)
    x = torch.randn(plan.grid_shape(), device="cuda", generator=gen)
    r = torch.randn(plan.grid_shape(), device="cuda", generator=gen)
    W = (torch.randn((L, C, C), device="cuda", generator=gen)
         + 1j * torch.randn((L, C, C), device="cuda", generator=gen)).to(torch.complex64) / (2 * C) ** 0.5
    y = torch.empty(plan.spec_shape(), dtype=torch.complex64, device="cuda")
    z, gz, gy = torch.empty_like(y), torch.empty_like(y), torch.empty_like(y)
    u, gx = torch.empty_like(x), torch.empty_like(x)
    dW = torch.empty_like(W)

    def step():
        plan.sht(x, out=y)
        plan.mix(W, y, out=z)
        plan.isht(z, out=u)
        plan.isht_T(r, out=gz)
        plan.mix(W, gz, adjoint=True, out=gy)
        plan.mix_weight_grad(gz, y, out=dW)
        plan.sht_T(gy, out=gx)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    plan.set_timing(True)
    plan.read_timing()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kt = plan.read_timing()
    plan.set_timing(False)
    avg = {k: 1000.0 * v[0] / v[1] for k, v in kt.items() if v[1]}
    mix_flops = 8.0 * C * C * sum(B * min(l + 1, L) for l in range(L))
    mix_us = avg.get("channel_mix", float("nan"))
    achieved = mix_flops / (mix_us * 1e-6) / 1e12
    peak = PEAKS_TFLOPS["fp32"]
    F = B * C
    out = {
        "metric": "spectral-convolution block fwd+bwd (SHT, per-degree channel mix, ISHT, adjoints, weight "
                  "gradient) fields/sec",
        "value": round(F * args.steps / wall, 1), "unit": "fields/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(wall * 1e3 / args.steps, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"Gauss 360x720, lmax=mmax=360, batch {B} x {C} channels; SHT -> mix_W -> ISHT "
                               "then ISHT^T -> mix_W^H and dW -> SHT^T",
                   "nlat": nlat, "nlon": nlon, "lmax": L, "mmax": L, "fields": F, "channels": C},
        "roofline": {"bound": "mfma", "kernel": "channel_mix (mix, mix^H, dW)", "achieved": round(achieved, 2),
                     "peak": peak, "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": None,
                     "avg_launch_us": round(mix_us, 2), "algorithmic_flops_per_launch": mix_flops},
        "cpu_baseline": None,
        "gpu_event_ms_per_step": round(e0.elapsed_time(e1) / args.steps, 4),
        "kernel_avg_us": {k: round(v, 2) for k, v in avg.items()},
    }
    print(json.dumps(out), flush=True)
    plan.close()


def scores_bench(args):
    """The consumers of the 721 x 1440 spectra: per step, for an ensemble of
    16 members x 8 channels, the spectral CRPS loss with its gradient
    (l <= 360, the paper's range), the angular PSD and the zonal PSD of every
    ring.  Roofline of the CRPS kernel against HBM: algorithmic bytes = the
    live coefficients (1 <= l <= 360, m <= l) of the ensemble and the
    observation read once, the full gradient tensor written once."""
    import numpy as np
    import torch
    import paper_2507_12144_amd as P
    torch.cuda.set_device(0)
    nlat, nlon, L, N, C = 721, 1440, 720, 16, 8
    plan = P.Plan(dict(nlat=nlat, nlon=nlon, lmax=L, mmax=L, grid="equiangular", batch=N, channels=C))
    gen = torch.Generator(device="cuda")
    gen.manual_seed(0)
    u = torch.randn(plan.grid_shape(), device="cuda", generator=gen)
    ens = plan.sht(u)
    obs = ens[0].clone()
    ens = ens + 0.1 * torch.randn(ens.shape, dtype=torch.complex64, device="cuda", generator=gen)
    g = torch.empty_like(ens)
    loss = torch.empty(C, device="cuda")
    psd = torch.empty((N, C, L), device="cuda")
    zpsd = torch.empty((N, C, nlat, L), device="cuda")
    lib = P._lib.load()
    import ctypes
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def step():
        P._lib.check(lib.sht_spectral_crps(plan._h, ctypes.c_void_p(ens.data_ptr()), ctypes.c_void_p(obs.data_ptr()),
                                           0, 0, ctypes.c_void_p(loss.data_ptr()), ctypes.c_void_p(g.data_ptr()), st))
        plan.psd(ens, out=psd)
        plan.zonal_psd(u, out=zpsd)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    plan.set_timing(True)
    plan.read_timing()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    plan.set_timing(False)
    kt = plan.read_timing()
    # per-kernel times from a separate timed pass of each (kind 6 covers all three)
    times = {}
    for name, fn in (("spectral_crps", lambda: P._lib.check(lib.sht_spectral_crps(
            plan._h, ctypes.c_void_p(ens.data_ptr()), ctypes.c_void_p(obs.data_ptr()), 0, 0,
            ctypes.c_void_p(loss.data_ptr()), ctypes.c_void_p(g.data_ptr()), st))),
                     ("psd", lambda: plan.psd(ens, out=psd)), ("zonal_psd", lambda: plan.zonal_psd(u, out=zpsd))):
        plan.set_timing(True)
        plan.read_timing()
        for _ in range(args.steps):
            fn()
        ms, n = plan.read_timing()["scores"]
        plan.set_timing(False)
        times[name] = 1000.0 * ms / n
    lhi = min(L - 1, nlat // 2)
    live = sum(min(l, L - 1) + 1 for l in range(1, lhi + 1))
    nbytes = (N + 1) * C * live * 8 + N * C * L * L * 8
    crps_us = times["spectral_crps"]
    achieved = nbytes / (crps_us * 1e-6) / 1e9
    out = {
        "metric": "spectral CRPS loss+gradient, angular PSD and zonal PSD fields/sec at 721x1440 lmax720",
        "value": round(N * C * args.steps / wall, 1), "unit": "fields/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(wall * 1e3 / args.steps, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "16 members x 8 channels, equiangular 721x1440, lmax=mmax=720: spectral CRPS "
                               "(l <= 360) with gradient, angular PSD, zonal PSD of every ring",
                   "members": N, "channels": C},
        "roofline": {"bound": "hbm", "kernel": "spectral_crps", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None, "avg_launch_us": round(crps_us, 2), "algorithmic_bytes_per_launch": nbytes},
        "cpu_baseline": None,
        "kernel_avg_us": {k: round(v, 2) for k, v in times.items()},
    }
    print(json.dumps(out), flush=True)
    plan.close()


def noise_bench(args):
    """The spherical diffusion noise of the paper's model input: 8 channels
    with the Table 1 length scales (lambda = 1, sigma = 1) for 16 ensemble
    members on the 721 x 1440 grid, lmax = mmax = 720; one step = one AR(1)
    update of every coefficient (Philox4x64-10 + Box-Muller in float64) and
    the ISHT of the new state."""
    import torch
    import paper_2507_12144_amd as P
    torch.cuda.set_device(0)
    nlat, nlon, L, B, C = 721, 1440, 720, 16, 8
    kT = [3.08e-5, 1.23e-4, 4.93e-4, 1.97e-3, 7.89e-3, 3.16e-2, 1.26e-1, 5.05e-1]
    plan = P.Plan(dict(nlat=nlat, nlon=nlon, lmax=L, mmax=L, grid="equiangular", batch=B, channels=C))
    noise = P.Noise(plan, kT, [1.0] * C, [1.0] * C, seed=2025)
    z = torch.empty(plan.grid_shape(), device="cuda")
    for _ in range(args.warmup):
        noise.step(out=z)
    torch.cuda.synchronize()
    plan.set_timing(True)
    plan.read_timing()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        noise.step(out=z)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kt = plan.read_timing()
    plan.set_timing(False)
    avg = {k: round(1000.0 * v[0] / v[1], 2) for k, v in kt.items() if v[1]}
    coeffs = B * C * L * L
    out = {
        "metric": "spherical diffusion noise fields/sec (AR(1) spectral step + ISHT) at 721x1440 lmax720",
        "value": round(B * C * args.steps / wall, 1), "unit": "fields/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(wall * 1e3 / args.steps, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "16 members x 8 Table-1 noise channels, equiangular 721x1440, lmax=mmax=720",
                   "members": B, "channels": C},
        "noise_step": {"avg_launch_us": avg.get("noise"), "coefficients": coeffs,
                       "gcoeff_per_s": round(coeffs / (avg.get("noise", float("nan")) * 1e-6) / 1e9, 2)},
        "cpu_baseline": None,
        "kernel_avg_us": avg,
    }
    print(json.dumps(out), flush=True)
    noise.close()
    plan.close()


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.workload in ("batched", "sfno_block", "scores", "noise"):
        if args.gpus != 1:
            print("bench.py measures one GPU only", file=sys.stderr, flush=True)
            sys.exit(2)
        {"batched": batched_bench, "sfno_block": sfno_block_bench, "scores": scores_bench,
         "noise": noise_bench}[args.workload](args)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); "
              "fields are independent, so N GPUs would each run this single-GPU workload.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    import paper_2507_12144_amd as P

    torch.cuda.set_device(0)
    nlat, nlon, L, M, B, C = 721, 1440, 720, 720, 1, 72
    F = B * C
    t0 = time.perf_counter()
    plan = P.Plan(dict(nlat=nlat, nlon=nlon, lmax=L, mmax=M, grid="equiangular", batch=B, channels=C),
                  precision=args.precision)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    tuned = None
    if args.schedule:
        plan.set_schedule(*[int(v) for v in args.schedule.split(",")])
    elif args.tune:
        choice, tune_ms = plan.tune(args.tune_cache)
        tuned = {"candidate": choice, "best_pass_ms": round(tune_ms, 3)}

    # synthetic input: band-limited field (seed 0) + 1e-3 white-noise probe (seed 1)
    a = torch.from_numpy(synth.coefficients(0, B, C, L, M).astype(np.complex64)).cuda()
    probe = torch.from_numpy(synth.white_noise(1, (B, C, nlat, nlon)).astype(np.float32)).cuda()
    u = plan.isht(a)
    u.add_(probe)
    del a, probe
    y = torch.empty(plan.spec_shape(), dtype=torch.complex64, device="cuda")
    x2 = torch.empty(plan.grid_shape(), dtype=torch.float32, device="cuda")
    gy = torch.empty_like(y)
    gx = torch.empty_like(x2)

    def step():
        plan.sht(u, out=y)
        plan.isht(y, out=x2)
        plan.isht_T(x2, out=gy)
        plan.sht_T(gy, out=gx)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # timed region: K eager steps, a HIP event pair around each (on the launch
    # stream) and around the whole region, plus per-kernel events inside
    plan.set_timing(True)
    plan.read_timing()
    stream = torch.cuda.current_stream()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record(stream)
    for i in range(args.steps):
        step()
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    plan.set_timing(False)
    kernels = plan.read_timing()
    gpu_ms = evs[0].elapsed_time(evs[-1])
    step_ms = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps)])
    ms_per_step = wall * 1e3 / args.steps
    value = F * args.steps / wall

    # the same four transforms captured as one HIP graph and replayed (outside
    # the timed region above; reported beside it)
    graph_ms = None
    if not args.profile_run:
        graph = plan.graph([("sht", u, y), ("isht", y, x2), ("isht_T", x2, gy), ("sht_T", gy, gx)])
        for _ in range(3):
            graph.launch()
        torch.cuda.synchronize()
        gev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        gev[0].record(stream)
        for i in range(args.steps):
            graph.launch()
            gev[i + 1].record(stream)
        torch.cuda.synchronize()
        graph_ms = np.array([gev[i].elapsed_time(gev[i + 1]) for i in range(args.steps)])
        graph.close()

    # roofline of the dominant kernel.  FP32: matrix-core bound, algorithmic
    # flops of the folded contraction.  bf16 forms: HBM bound, algorithmic
    # bytes = the folded table in its storage form + the dense spectrum.
    ana_ms, ana_n = kernels["legendre_analysis"]
    syn_ms, syn_n = kernels["legendre_synthesis"]
    # a staged analysis is charged with its spectrum transpose, a staged
    # synthesis input with its staging kernel
    tr_ms, tr_n = kernels.get("transpose", (0.0, 0))
    if tr_n:
        ana_ms += tr_ms * ana_n / tr_n
    sg_ms, sg_n = kernels.get("stage", (0.0, 0))
    if sg_n:
        syn_ms += sg_ms * syn_n / sg_n
    kind, tot, n = ("legendre_analysis", ana_ms, ana_n) if ana_ms >= syn_ms else ("legendre_synthesis", syn_ms, syn_n)
    extra = (" + spectrum transpose" if tr_n and kind == "legendre_analysis" else
             " + input staging" if sg_n and kind == "legendre_synthesis" else "")
    flops = legendre_flops(nlat, L, M, F)
    nbytes = legendre_bytes(nlat, L, M, F, args.precision)
    avg_s = tot / max(n, 1) * 1e-3
    if args.precision == "fp32":
        achieved, peak = flops / avg_s / 1e12, PEAKS_TFLOPS["fp32"]
        roofline = {"bound": "mfma", "kernel": kind + extra, "achieved": round(achieved, 2), "peak": peak,
                    "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": None,
                    "avg_launch_us": round(avg_s * 1e6, 2), "algorithmic_flops_per_launch": flops}
        step_bound_ms = 4 * flops / (peak * 1e12) * 1e3
    else:
        achieved, peak = nbytes / avg_s / 1e9, HBM_PEAK_GBS
        roofline = {"bound": "hbm", "kernel": kind + extra, "achieved": round(achieved, 1), "peak": peak,
                    "unit": "GB/s", "frac": round(achieved / peak, 4), "traffic": None,
                    "avg_launch_us": round(avg_s * 1e6, 2), "algorithmic_bytes_per_launch": nbytes,
                    "mfma_tflops": round(flops * PRODUCTS[args.precision] / avg_s / 1e12, 2)}
        step_bound_ms = 4 * nbytes / (peak * 1e9) * 1e3
    p50 = float(np.percentile(step_ms, 50))
    # the whole step against the sum of its dominant-kernel bounds (four
    # Legendre launches; the ring DFTs and everything else count as overhead)
    roofline["step_frac"] = round(step_bound_ms / p50, 4)
    # the same fraction against the peaks measured on this GPU (a streaming
    # copy, matrix-core loops)
    peaks = None
    if not args.profile_run:
        peaks = P.measure_peaks()
        roofline["peak_measured"] = peaks["fp32_mfma_TFs"] if args.precision == "fp32" else peaks["hbm_measured_GBs"]
        roofline["frac_measured"] = round(achieved / roofline["peak_measured"], 4)
    prof = profiled_traffic(kind, args.precision,
                            "spectrum_transpose" if extra == " + spectrum transpose" else
                            "spectrum_stage" if extra == " + input staging" else None)
    if prof is not None:
        roofline["traffic"] = prof["hbm_bytes_per_launch"]
        roofline["traffic_unit"] = "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
        roofline["traffic_source"] = prof["source"]
    per_kernel_us = {k: round(v[0] / max(v[1], 1) * 1e3, 2) for k, v in kernels.items() if v[1]}

    # CPU baseline: the FP64 oracle doing the same four transforms on the host
    # (each stage fed the GPU stage's input, so the same pass also gives every
    # stage's error); one untimed warm-up pass, then the median of three.  The
    # oracle rebuilds each order's Legendre rows inside every transform; that
    # recurrence is timed on its own and reported separately.
    err = None
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        from oracle.legendre import iter_orders
        try:
            from threadpoolctl import threadpool_info
            blas_threads = max([i.get("num_threads", 0) for i in threadpool_info()] or [0])
        except Exception:
            blas_threads = 0
        nf = max(1, min(args.cpu_fields, F))
        ins = [t.cpu().numpy()[:, :nf] for t in (u, y, x2, gy)]
        outs = [t.cpu().numpy()[:, :nf] for t in (y, x2, gy, gx)]
        u_h, y_h, x_h, gy_h = ins[0].astype(np.float64), ins[1].astype(np.complex128), \
            ins[2].astype(np.float64), ins[3].astype(np.complex128)

        def cpu_pass():
            return (oracle.sht(u_h, L, M, 0), oracle.isht(y_h, nlat, nlon, 0),
                    oracle.isht_T(x_h, L, M, 0), oracle.sht_T(gy_h, nlat, nlon, 0))

        refs = cpu_pass()                      # warm-up
        times = []
        for _ in range(3):
            t0 = time.perf_counter()
            cpu_pass()
            times.append(time.perf_counter() - t0)
        th, xk, _ = oracle.grid(nlat, 0)
        t0 = time.perf_counter()
        for _m, _rows in iter_orders(L, M, xk, np.sin(th)):
            pass
        table_s = time.perf_counter() - t0
        med = float(np.median(times))
        err = {name: float(np.linalg.norm((got - ref).ravel()) / np.linalg.norm(ref.ravel()))
               for name, got, ref in zip(("sht", "isht", "isht_T", "sht_T"), outs, refs)}
        cpu = {"value": round(nf / max(med - 4 * table_s, 1e-9), 3), "unit": "fields/s",
               "cores": blas_threads or os.cpu_count(), "kind": "oracle",
               "value_incl_table": round(nf / med, 3),
               "sample": f"{nf} of the {F} fields, full 721x1440 grid: SHT, ISHT, ISHT^T, SHT^T in float64; median "
                         f"of 3 passes after 1 warm-up ({med:.2f} s per pass), minus the oracle's own Legendre "
                         f"recurrence (4 x {table_s:.2f} s per pass, reported as table_build_s); "
                         f"os.cpu_count()={os.cpu_count()}, affinity={len(os.sched_getaffinity(0))}",
               "table_build_s": round(table_s, 3)}

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "fields/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32" if args.precision == "fp32" else args.precision,
        "data": "synthetic",
        "config": {"workload": "SHT->ISHT->ISHT^T->SHT^T, equiangular 721x1440 with poles (Clenshaw-Curtis), "
                               "lmax=mmax=720, batch 1 x 72 channels",
                   "nlat": nlat, "nlon": nlon, "lmax": L, "mmax": M, "fields": F, "precision": args.precision},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "err_vs_fp64": err,
        "gpu_event_ms_per_step": round(gpu_ms / args.steps, 4),
        "step_ms": {"p10": round(float(np.percentile(step_ms, 10)), 4), "p50": round(p50, 4),
                    "p90": round(float(np.percentile(step_ms, 90)), 4)},
        "graph_replay_ms": None if graph_ms is None else {
            "p10": round(float(np.percentile(graph_ms, 10)), 4), "p50": round(float(np.percentile(graph_ms, 50)), 4),
            "p90": round(float(np.percentile(graph_ms, 90)), 4)},
        "kernel_avg_us": per_kernel_us,
        "plan_build_s": round(plan_s, 3),
    }
    print(json.dumps(out), flush=True)
    plan.close()


if __name__ == "__main__":
    main()
