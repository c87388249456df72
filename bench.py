#!/usr/bin/env python3
"""Benchmark of the distributed-MIMO hot path on one MI355X.

Workload ("room"): M = 64 APs on a jittered 8x8 ceiling grid (pitch 2.5 m,
z = 4 m) of a 20x20x4 m room, 3.5 GHz, K = 8 users at z = 1.2 m, noise -90 dBm.
One step is one pass of the whole path, with inputs already resident in HBM:

  1. dmimo_beamform_users  user channels H (K x M, complex64, synthesised in
                           the launch and written out), and MR and ZF of them
                           at 1 W (+ p_m, L2,1, SINR_k, R_sum) in one launch;
                           ZF with its FP64 Gram and inverse
  2. dmimo_powermap_batch  MR and ZF power + SINR + best-stream maps, 512 x 512
                           grid at z = 1.2 m, both maps in one launch

value = channel terms h[n,m] synthesised and consumed per second, over the
whole step (K M for the channels and for each precoder, N M for each map), in
G h/s.  The timed steps rotate over two HIP streams (--streams): each step is
an independent pass with its own outputs, so one stream's precoder launch and
its map launch's ramp and drain overlap the other stream's map.  The JSON
line's ``one_stream`` gives the same steps on a single stream, and the
roofline's map launch duration is measured on a single stream.

The JSON line also carries:
* ``roofline`` for the dominant kernel (the FP32 power map).  It is bound by
  plain VALU arithmetic; the algorithmic cost and the peak are stated below.
* ``cpu_baseline``: the FP64 oracle timed on a bounded sample of the same step.
* ``err_db``: the error of the GPU maps against the oracle on that sample.

Only the cpu_baseline leg imports the oracle.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# ---------------------------------------------------------------------------
# roofline model of the power-map kernel (VALU issue slots)
# ---------------------------------------------------------------------------
# MI355X: 256 CUs x 4 SIMDs x 16 lanes per clock x 2.4 GHz = 39.3e12 lane-slots/s.
# FP64 add/mul/FMA and unpacked FP32 ops issue at that full rate.  The
# transcendental ops (rsq, sin, cos) take 4 slots each.
VALU_PEAK_SLOTS = 256 * 4 * 16 * 2.4e9
# Algorithmic slots per term for FP64 distance/phase + FP32 synthesis:
#   3 sub + 3 (mul, 2 FMA) for d^2                             6
#   sqrt: cvt, rsq(4), cvt, 4 FP64 Newton ops                  10
#   revolutions: mul, floor, FMA (fract), cvt                   4
#   sin(4) + cos(4)                                             8
#   amplitude min + mul, h = amp * (c, -s): 2 mul                4
# = 32 slots.  With K >= 3 the K complex MACs (8K real flops per term) run on
# FP32 MFMA (157.3 TFLOP/s dense) and overlap the VALU; the kernel is bound by
# whichever of the two pipes has the larger fraction.
SYNTH_SLOTS = 32
MFMA_F32_PEAK = 157.3e12


def alg_slots_per_term(K: int) -> int:
    return SYNTH_SLOTS if K >= 3 else SYNTH_SLOTS + 4 * K


def _src_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


# every file the map kernels are compiled from (the traffic summary is only
# valid for these exact sources)
POWERMAP_SOURCES = ["paper_2304_12745_amd/csrc/powermap.hip",
                    "paper_2304_12745_amd/csrc/powermap_mfma.hip",
                    "paper_2304_12745_amd/csrc/powermap_mfma.h",
                    "paper_2304_12745_amd/csrc/powermap_body.h",
                    "paper_2304_12745_amd/csrc/powermap_common.h",
                    "paper_2304_12745_amd/csrc/split16.h",
                    "paper_2304_12745_amd/csrc/kernels.h",
                    "paper_2304_12745_amd/csrc/dmimo_internal.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "powermap_room_traffic.json")


def load_traffic(kernel_hash: str):
    """HBM bytes per launch from the committed rocprofv3 --pmc summary.

    None if there is none, or if it was taken on other kernel sources.
    """
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != kernel_hash:
        return None
    return t.get("bytes_per_launch")


def parse_args():
    p = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=500)
    p.add_argument("--warmup", type=int, default=2000,
                   help="untimed steps first (enough to bring the GPU clocks up)")
    p.add_argument("--event-every", type=int, default=10,
                   help="record the map event pair on every n-th timed step (each pair "
                        "puts two markers in the queue, about 7 us per step)")
    p.add_argument("--nx", type=int, default=512)
    p.add_argument("--streams", type=int, default=2,
                   help="HIP streams the timed steps rotate over (independent steps, each "
                        "stream with its own outputs); 1 = every step on one stream")
    p.add_argument("--cpu-seconds", type=float, default=10.0,
                   help="budget of the oracle CPU baseline (0 disables it)")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--serve-seconds", type=float, default=5.0,
                   help="measured window of the serving phase (0 disables it)")
    p.add_argument("--serve-warmup", type=float, default=1.0)
    p.add_argument("--serve-rate", type=float, default=2000.0, help="Poisson arrival rate (1/s)")
    p.add_argument("--serve-prec", default="f32", choices=["f32", "f16x3", "bf16x3"])
    p.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision step")
    p.add_argument("--no-pgd", action="store_true", help="skip the PGD / unfolded-PGD phase")
    p.add_argument("--no-pa", action="store_true", help="skip the PA-aware precoder phase")
    p.add_argument("--no-channel", action="store_true",
                   help="skip the materialised-channel bandwidth phase")
    p.add_argument("--no-batched", action="store_true",
                   help="skip the batched Gram + ZF sweep over B")
    p.add_argument("--serve-sweep", action="store_true",
                   help="also serve at 500, 1000, 2000 and 4000 queries/s (3 s each)")
    return p.parse_args()


def main():
    args = parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(the grid points of a map would shard across GPUs with no exchange).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2304_12745_amd import dmimo as D
    from paper_2304_12745_amd import workloads as WL

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    D.lib()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    w = WL.room_workload(nx=args.nx, ny=args.nx)
    K, M, N = w.K, w.M, w.grid.n
    params = D.channel_params(w.freq_hz)
    ap = torch.from_numpy(w.ap_xyz).to(dev)            # [1][M][3]
    ap0 = ap[0].contiguous()
    users = torch.from_numpy(w.user_xyz).to(dev)       # [1][K][3]
    gpts = D.grid_points(w.grid)
    H = torch.empty((1, K, M), dtype=torch.complex64, device=dev)

    # a plain copy of known size, for scaling the HBM counters of a profiled run
    cp_src = torch.empty(64 << 20, dtype=torch.uint8, device=dev)
    cp_dst = torch.empty_like(cp_src)
    cp_dst.copy_(cp_src)

    # one stream: the map launch's own duration (HIP events) for the roofline
    ms_one, map_launch_ms, maps, bf = run_steps(args, "f32", w, D, params, ap, ap0, users,
                                                gpts, H)
    ms_per_step = ms_one
    if args.streams > 1:
        # the headline: steps in flight on args.streams streams
        ms_per_step = run_steps(args, "f32", w, D, params, ap, ap0, users, gpts, H,
                                nstreams=args.streams)[0]
    mixed = None
    if not args.no_mixed:
        ms_mix, launch_mix, maps_mix, _ = run_steps(args, "f16x3", w, D, params, ap, ap0, users,
                                                    gpts, H)
        dev_db = {}
        for p in ("mr", "zf"):
            a = maps_mix[p].power.double()
            b = maps[p].power.double()
            keep = b > 1e-6 * b.max()     # the -60 dB floor of the error rule
            dev_db[p] = float((10 * torch.log10(a[keep] / b[keep])).abs().max())
        ms_mix_n = None
        if args.streams > 1:
            ms_mix_n = round(run_steps(args, "f16x3", w, D, params, ap, ap0, users, gpts, H,
                                       nstreams=args.streams)[0], 5)
        mixed = {"dtype": "f16x3 (FP16 hi/lo x3 MFMA, FP32 accumulate)", "streams": 1,
                 "ms_per_step": round(ms_mix, 5), "maps_launch_ms": round(launch_mix, 5),
                 "speedup_vs_f32_step": round(ms_one / ms_mix, 3),
                 "ms_per_step_streams": ms_mix_n,
                 "max_db_vs_f32_maps": dev_db}

    terms_per_step = 3 * K * M + 2 * N * M
    value = terms_per_step / (ms_per_step * 1e-3) / 1e9
    terms_per_launch = 2 * N * M          # both maps in one launch
    alg = alg_slots_per_term(K) * terms_per_launch
    achieved = alg / (map_launch_ms * 1e-3) / 1e12
    peak = VALU_PEAK_SLOTS / 1e12
    mfma_tflops = 8 * K * terms_per_launch / (map_launch_ms * 1e-3) / 1e12
    khash = _src_hash(POWERMAP_SOURCES)
    traffic = load_traffic(khash)

    out = {
        "metric": "channel-term evals/sec (G h[n,m]/s)",
        "value": round(value, 3),
        "unit": "G h/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "streams": args.streams,
        "one_stream": {"ms_per_step": round(ms_one, 5),
                       "value": round(terms_per_step / (ms_one * 1e-3) / 1e9, 3)},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"room: M={M} APs jittered 8x8 ceiling grid 20x20x4 m, K={K} users, "
                        f"3.5 GHz, MR+ZF at 1 W, noise -90 dBm, {w.grid.nx}x{w.grid.ny} power+SINR "
                        "maps at z=1.2 m; FP64 distance/phase, FP32 synthesis and contraction",
            "M": M, "K": K, "N": N, "terms_per_step": terms_per_step,
        },
        "roofline": {
            "bound": "alu",
            "kernel": "powermap_mfma_kernel<1,4,8>, grid 512 x 2 (MR and ZF maps in one launch)",
            "achieved": round(achieved, 3),
            "peak": round(peak, 3),
            "unit": "T VALU lane-slots/s",
            "frac": round(achieved / peak, 4),
            "traffic": traffic,
            "launch_ms": round(map_launch_ms, 5),
            "event_samples": len(range(0, args.steps, max(1, args.event_every))),
            "alg_slots_per_term": alg_slots_per_term(K),
            "mfma_f32": {"achieved": round(mfma_tflops, 3), "peak": MFMA_F32_PEAK / 1e12,
                         "unit": "TFLOP/s", "frac": round(mfma_tflops * 1e12 / MFMA_F32_PEAK, 4),
                         "flops_per_term": 8 * K},
            # the matrix unit and the VALU do not co-issue on this kernel
            # (SQ_VALU_MFMA_COEXEC_CYCLES = 0), so its floor is the sum of the
            # synthesis at the VALU peak and the contraction at the MFMA peak
            "serial_valu_mfma": {
                "floor_ms": round((alg / VALU_PEAK_SLOTS + 8 * K * terms_per_launch / MFMA_F32_PEAK)
                                  * 1e3, 5),
                "frac": round((alg / VALU_PEAK_SLOTS + 8 * K * terms_per_launch / MFMA_F32_PEAK) * 1e3
                              / map_launch_ms, 4)},
            "terms_per_launch": terms_per_launch,
            "source_hash": khash,
        },
    }

    if mixed is not None:
        mixed["value"] = round(terms_per_step / (mixed["ms_per_step"] * 1e-3) / 1e9, 3)
        out["mixed"] = mixed
    if not args.no_channel:
        out["channel"] = channel_phase(D, WL, torch, params, ap, gpts, N)
    if not args.no_batched:
        out["batched"] = batched_phase(D, torch)
    if args.serve_seconds > 0:
        out["serving"] = serving_phase(args, D, WL, torch)
    if args.serve_sweep:
        sweep = []
        for rate in (500.0, 1000.0, 2000.0, 4000.0):
            a2 = argparse.Namespace(**vars(args))
            a2.serve_rate, a2.serve_seconds = rate, 3.0
            r = serving_phase(a2, D, WL, torch)
            sweep.append({k: r[k] for k in ("rate_qps", "queries", "p50_ms", "p99_ms", "max_ms",
                                            "sustained_Gh_per_s", "offered_Gh_per_s")})
        out["serving_sweep"] = sweep
    if not args.no_pgd:
        out["pgd"] = pgd_phase(args, D, WL, torch)
    if not args.no_pa:
        out["pa"] = pa_phase(w, D, WL, torch, params, ap0, gpts)
    if not args.no_cpu and args.cpu_seconds > 0:
        out["cpu_baseline"], out["err_db"] = cpu_baseline(w, bf, maps, args.cpu_seconds)

    print(json.dumps(out), flush=True)


def run_steps(args, prec, w, D, params, ap, ap0, users, gpts, H, nstreams=1):
    """Warm up, then time exactly args.steps steps of the room workload.

    With nstreams > 1, step i runs on stream i % nstreams, each stream with
    its own H, precoder and map outputs, and no step waits for another: the
    steps are independent passes, so one stream's precoder launch (two
    workgroups) and its map launch's ramp and drain overlap another stream's
    map.  No events are recorded then; the launch figure is None.

    One step, in order on torch's current stream: the user channels and the
    MR and ZF precoders of those channels (Gram and inverse inside) in one
    dmimo_beamform_users launch, H written to ``H`` and W into one [2][K][M]
    array; the MR and ZF maps in one dmimo_powermap_batch launch (map p on
    grid row p).  One pair of HIP events on that stream brackets the map
    launch of every args.event_every-th timed step (a pair on every step
    adds about 7 us per step).  (A variant with the MR branch on a second
    stream was measured slower: 0.114 vs 0.094 ms/step, because the
    cross-queue event waits cost more than the overlap saves.)
    Returns (ms per step, mean ms of the two-map launch, maps per precoder,
    precoders).
    """
    import torch
    K, M, N = w.K, w.M, w.grid.n
    dev = H.device
    if nstreams > 1:
        return run_streams(args, prec, w, D, params, ap, ap0, users, gpts, nstreams)
    both = D.MapResult(torch.empty((2, N), device=dev), torch.empty((2, N), device=dev),
                       torch.empty((2, N), dtype=torch.int32, device=dev), None)
    maps = {p: D.MapResult(both.power[i], both.sinr[i], both.best_k[i], None)
            for i, p in enumerate(("mr", "zf"))}
    pcs = ("mr", "zf")
    pre = D.beamform_users(params, ap, users, pcs, None, w.sigma2, w.p_total, prec,
                           H=H)                                     # outputs [2][1][...]
    Wst = pre.W.view(2, K, M)
    bf = {p: D.BeamformResult(pre.W[i], pre.p_ant[i], pre.l21[i], pre.sinr[i], pre.rsum[i],
                              pre.info[i]) for i, p in enumerate(pcs)}

    def step(e=None):
        D.beamform_users(params, ap, users, pcs, None, w.sigma2, w.p_total, prec, out=pre)
        if e is not None:
            e[0].record()
        D.powermap_batch(params, ap0, Wst, gpts, w.sigma2, prec, out=both)
        if e is not None:
            e[1].record()

    for _ in range(args.warmup):
        step()
    every = max(1, args.event_every)
    events = {i: [torch.cuda.Event(enable_timing=True) for _ in range(2)]
              for i in range(0, args.steps, every)}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(events.get(i))
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    launch = sum(e[0].elapsed_time(e[1]) for e in events.values()) / len(events)
    return ms, launch, maps, bf


def run_streams(args, prec, w, D, params, ap, ap0, users, gpts, nstreams):
    """run_steps over nstreams streams (default priority), step i on stream
    i % nstreams.  Every stream's maps are checked equal to stream 0's after
    the timed steps.  Returns (ms per step, None, None, None)."""
    import torch
    K, M, N = w.K, w.M, w.grid.n
    dev = ap.device
    pcs = ("mr", "zf")
    streams = [torch.cuda.Stream(device=dev) for _ in range(nstreams)]
    bufs = []
    torch.cuda.synchronize()
    for s in streams:
        H = torch.empty((1, K, M), dtype=torch.complex64, device=dev)
        pre = D.beamform_users(params, ap, users, pcs, None, w.sigma2, w.p_total, prec, H=H,
                               stream=s)
        both = D.MapResult(torch.empty((2, N), device=dev), torch.empty((2, N), device=dev),
                           torch.empty((2, N), dtype=torch.int32, device=dev), None)
        bufs.append((s, pre, pre.W.view(2, K, M), both))
    torch.cuda.synchronize()

    def step(i):
        s, pre, Wst, both = bufs[i % nstreams]
        D.beamform_users(params, ap, users, pcs, None, w.sigma2, w.p_total, prec, out=pre,
                         stream=s)
        D.powermap_batch(params, ap0, Wst, gpts, w.sigma2, prec, out=both, stream=s)

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(i)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    for _, _, _, both in bufs[1:]:
        if not (torch.equal(both.power, bufs[0][3].power) and torch.equal(both.sinr, bufs[0][3].sinr)):
            raise RuntimeError("maps differ between streams")
    return ms, None, None, None


HBM_PEAK = 8.0e12   # MI355X HBM3E, bytes/s


def channel_phase(D, WL, torch, params, ap, gpts, N):
    """dmimo_channel materialising H in HBM, an HBM-write-bound kernel: the
    room grid (512 x 512 points x 64 APs) in complex64 and complex128, and the
    hall grid (2048 x 2048 points x 1024 APs, 34.4 GB) in complex64.  Kernel
    time from HIP events around back-to-back launches; bytes = the output."""
    def run(prm, apd, pts, n, m, prec, reps):
        H = D.channel(prm, apd, pts, prec=prec)
        for _ in range(2):
            D.channel(prm, apd, pts, prec=prec, out=H)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            D.channel(prm, apd, pts, prec=prec, out=H)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        del H
        torch.cuda.empty_cache()
        nbytes = n * m * (16 if prec == "f64" else 8)
        return {"ms": round(ms, 4), "G_h_per_s": round(n * m / ms / 1e6, 1),
                "GB_per_s": round(nbytes / ms / 1e6, 1), "hbm_frac": round(nbytes / (ms * 1e-3) / HBM_PEAK, 3)}
    M = ap.shape[1]
    out = {"room_f32": run(params, ap, gpts, N, M, "f32", 50),
           "room_f64": run(params, ap, gpts, N, M, "f64", 50)}
    hw = WL.hall_workload()
    hap = torch.from_numpy(hw.ap_xyz).to(ap.device)
    out["hall_f32"] = run(D.channel_params(hw.freq_hz), hap, D.grid_points(hw.grid), hw.grid.n,
                          hw.M, "f32", 5)
    out["workload"] = ("room: 512 x 512 grid x 64 APs (16.8 M terms); hall: 2048 x 2048 grid x "
                       "1024 APs (4.29 G terms); LoS, output H [N][M] in HBM")
    return out


def batched_phase(D, torch):
    """Batched Gram + ZF (dmimo_beamform at 1 W, -90 dBm) on B deployments of
    K = 16 users and M = 256 antennas, B = 2^10 .. 2^17, with the FP32 and
    the FP16x3 Gram.  The cost does not depend on the channel values, so H is
    CN(0,1), drawn on the device by torch with a fixed seed.  Units: B K M
    terms per call; time from HIP events around back-to-back calls."""
    K, M = 16, 256
    gen = torch.Generator(device="cuda")
    gen.manual_seed(3)
    bmax = 1 << 17
    H = torch.complex(torch.randn(bmax, K, M, generator=gen, device="cuda"),
                      torch.randn(bmax, K, M, generator=gen, device="cuda")) * (0.5 ** 0.5)
    sweep = []
    for prec in ("f32", "f16x3"):
        for e in (10, 12, 14, 16, 17):
            B = 1 << e
            Hb = H[:B]
            r = D.beamform(Hb, "zf", None, 1e-12, 1.0, prec)
            reps = 20 if B <= 1 << 14 else 5
            for _ in range(2):
                D.beamform(Hb, "zf", None, 1e-12, 1.0, prec, out=r)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(reps):
                D.beamform(Hb, "zf", None, 1e-12, 1.0, prec, out=r)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            sweep.append({"B": B, "prec": prec, "ms": round(ms, 4),
                          "deployments_per_s": round(B / ms * 1e3, 1),
                          "G_h_per_s": round(B * K * M / ms / 1e6, 2)})
            del r
    del H
    torch.cuda.empty_cache()
    return {"workload": "batched ZF: B deployments x K=16 users x M=256 antennas, H ~ CN(0,1) "
                        "(device draws), total power 1 W, noise -90 dBm; Gram + inverse + W + epilogues",
            "sweep": sweep}


def serving_phase(args, D, WL, torch):
    """Poisson stream of power-map queries (M in {16,64,256,512}, N in
    {64^2,256^2,1024^2}, K in {1,4,16}, f in {0.92,3.5,5.8} GHz, MR/ZF) into a
    dmimo server with resident geometry.  Latency = completion - arrival."""
    import numpy as np
    pool = WL.serving_pool()
    total_s = args.serve_warmup + args.serve_seconds
    n_q = int(args.serve_rate * total_s * 1.2) + 16
    qs = WL.serving_queries(pool, n_q, rate_hz=args.serve_rate)
    qs = [q for q in qs if q.t_arrival < total_s]
    dev = torch.device("cuda")
    srv = D.Server(16 << 30, 64)
    deps = [srv.add_deployment(D.channel_params(f), aps) for (M, f, aps) in pool]
    # output buffers per grid side, recycled after completion
    free = {s: [] for s in WL.SERVE_SIDE}
    def get_buf(side):
        if free[side]:
            return free[side].pop()
        n = side * side
        return (torch.empty(n, device=dev), torch.empty(n, device=dev))
    for side, cnt in ((64, 64), (256, 64), (1024, 64)):
        free[side] = [(torch.empty(side * side, device=dev), torch.empty(side * side, device=dev))
                      for _ in range(cnt)]
    torch.cuda.synchronize()
    outstanding = []          # (ticket, query, buf)
    done = []                 # (arrival_abs, t_done, terms, measured)
    t0 = time.monotonic() + 0.05
    sigma2 = WL.NOISE_MINUS_90_DBM_W

    def reap(block_one=False):
        keep = []
        for i, (tk, q, buf, ta) in enumerate(outstanding):
            st, _, td = srv.poll(tk)
            if st >= D.Q_DONE:
                done.append((ta, td, q.M * q.side * q.side, q.t_arrival >= args.serve_warmup, st))
                srv.release(tk)
                free[q.side].append(buf)
            else:
                keep.append((tk, q, buf, ta))
        outstanding[:] = keep

    for q in qs:
        ta = t0 + q.t_arrival
        while True:
            now = time.monotonic()
            if now >= ta:
                break
            if ta - now > 2e-4 and outstanding:
                reap()
        buf = get_buf(q.side)
        tk = srv.submit(deps[q.dep], q.user_xyz, q.precoder, D.grid_points(q.grid), sigma2, 1.0,
                        args.serve_prec, buf[0], buf[1])
        outstanding.append((tk, q, buf, ta))
    while outstanding:
        tk = outstanding[0][0]
        srv.wait(tk, 30.0)
        reap()
    stats = srv.stats()
    srv.close()
    meas = [d for d in done if d[3]]
    lat = np.array([d[1] - d[0] for d in meas]) * 1e3
    failed = sum(1 for d in done if d[4] != D.Q_DONE)
    t_first = min(d[0] for d in meas)
    t_last = max(d[1] for d in meas)
    terms = sum(d[2] for d in meas)
    offered = sum(q.M * q.side * q.side for q in qs if q.t_arrival >= args.serve_warmup)
    return {
        "workload": "Poisson 2000 q/s power maps: M in {16,64,256,512}, N in {64^2,256^2,1024^2}, "
                    "K in {1,4,16}, f in {0.92,3.5,5.8} GHz, MR/ZF; geometry resident",
        "prec": args.serve_prec,
        "rate_qps": args.serve_rate,
        "measured_s": args.serve_seconds,
        "queries": len(meas),
        "failed": failed,
        "p50_ms": round(float(np.percentile(lat, 50)), 3),
        "p99_ms": round(float(np.percentile(lat, 99)), 3),
        "max_ms": round(float(lat.max()), 3),
        "sustained_Gh_per_s": round(terms / (t_last - t_first) / 1e9, 2),
        "offered_Gh_per_s": round(offered / args.serve_seconds / 1e9, 2),
        "launches": stats["launches"],
    }


def pgd_phase(args, D, WL, torch):
    """The paper's solver on its own workload (Sec. VI): 5000 Rayleigh channels
    H ~ CN(0, 1), K = 8, M = 64, gamma = 10 dB, sigma = 1, W(0) = H^*.

    * UfPGD inference, 20 layers (one dmimo_pgd launch over all channels);
    * PGD, 5000 iterations, lambda = 1/15, eta = 1/L~ (the paper's reference
      solution), with its mean PCG against ZF and sum rate;
    * ZF with the paper's scaling (the PCG reference), dmimo_beamform;
    * one training step of the unfolded network (batch 64, 20 layers, forward
      + reverse pass + Adam), dmimo_ufpgd_train;
    * the FP64 oracle's UfPGD inference, single-threaded, on a sample.
    HIP events on the launching stream time every call.  The roofline is that
    of pgd_mfma_kernel: 16 K^2 M real flops per layer and channel (the two
    complex K x K x M products of the layer) on FP32 MFMA."""
    import math

    import numpy as np

    K, M, B, I = 8, 64, 5000, 20
    L = (math.sqrt(K) + math.sqrt(M)) ** 2
    w = WL.paper_workload(seed=0, B=B)
    H = torch.from_numpy(w.H.astype(np.complex64)).cuda()
    g = w.gamma_lin

    def timed(fn, reps, warm=2):
        for _ in range(warm):
            fn()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * reps)]
        torch.cuda.synchronize()
        for r in range(reps):
            ev[2 * r].record()
            fn()
            ev[2 * r + 1].record()
        torch.cuda.synchronize()
        return sum(ev[2 * r].elapsed_time(ev[2 * r + 1]) for r in range(reps)) / reps

    lam20 = torch.full((I,), 1.0 / 15.0, dtype=torch.float64, device="cuda")
    eta20 = torch.full((I,), 1.0 / L, dtype=torch.float64, device="cuda")
    out20 = D.pgd(H, lam20, eta20, g, 1.0)
    ms20 = timed(lambda: D.pgd(H, lam20, eta20, g, 1.0, out=out20), 50)
    lam5k = torch.full((5000,), 1.0 / 15.0, dtype=torch.float64, device="cuda")
    eta5k = torch.full((5000,), 1.0 / L, dtype=torch.float64, device="cuda")
    out5k = D.pgd(H, lam5k, eta5k, g, 1.0)
    ms5k = timed(lambda: D.pgd(H, lam5k, eta5k, g, 1.0, out=out5k), 3, warm=1)
    zf = D.beamform(H, "zf", g, 1.0, 0.0, "f32")
    mszf = timed(lambda: D.beamform(H, "zf", g, 1.0, 0.0, "f32", out=zf), 20)
    pcg5k = (zf.l21 / out5k.l21).mean().item()
    # the same two launches with BF16x3 layers (split products on BF16 MFMA)
    x20 = D.pgd(H, lam20, eta20, g, 1.0, prec="bf16x3")
    ms20_x3 = timed(lambda: D.pgd(H, lam20, eta20, g, 1.0, prec="bf16x3", out=x20), 50)
    x5k = D.pgd(H, lam5k, eta5k, g, 1.0, prec="bf16x3")
    ms5k_x3 = timed(lambda: D.pgd(H, lam5k, eta5k, g, 1.0, prec="bf16x3", out=x5k), 3, warm=1)
    pcg5k_x3 = (zf.l21 / x5k.l21).mean().item()

    Htr = torch.from_numpy(WL.complex_normal(np.random.default_rng(9), (20000, K, M),
                                             np.complex64)).cuda()
    st = D.UfpgdState([1.0 / 15.0] * I, [1.0 / L] * I, torch.device("cuda"))
    rng = np.random.default_rng(10)
    steps = 300
    idx = torch.from_numpy(np.stack([rng.permutation(20000)[:64] for _ in range(steps)])
                           .astype(np.int32)).cuda()
    ws = torch.empty((D.ufpgd_workspace_size(64, K, M, I),), dtype=torch.uint8, device="cuda")
    ms_train = timed(lambda: D.ufpgd_train(Htr, st, idx, g, 1.0, ws=ws), 3, warm=1) / steps

    flops20 = 16 * K * K * M * I * B
    achieved = flops20 / (ms20 * 1e-3) / 1e12
    res = {
        "workload": f"paper: {B} Rayleigh channels CN(0,1), K={K}, M={M}, gamma 10 dB, sigma 1",
        "ufpgd20_ms": round(ms20, 4),
        "ufpgd20_channels_per_s": round(B / (ms20 * 1e-3)),
        "pgd5000_ms": round(ms5k, 3),
        "pgd5000_mean_pcg": round(pcg5k, 4),
        "pgd5000_mean_rsum": round(out5k.rsum.mean().item(), 4),
        "zf_ms": round(mszf, 4),
        "bf16x3": {"ufpgd20_ms": round(ms20_x3, 4), "pgd5000_ms": round(ms5k_x3, 3),
                   "pgd5000_mean_pcg": round(pcg5k_x3, 4),
                   "note": "both products of every layer on BF16 MFMA, operands split hi + lo, "
                           "three products accumulated in FP32"},
        "train_step_ms": round(ms_train, 4),
        "train_step": "batch 64, 20 layers: forward + reverse pass + Adam + projections",
        "roofline": {"bound": "mfma", "kernel": "pgd_mfma_kernel", "unit": "TFLOP/s",
                     "achieved": round(achieved, 3), "peak": MFMA_F32_PEAK / 1e12,
                     "frac": round(achieved * 1e12 / MFMA_F32_PEAK, 4),
                     "flops_per_launch": flops20, "launch_ms": round(ms20, 4),
                     "pgd5000_frac": round(16 * K * K * M * 5000 * B / (ms5k * 1e-3)
                                           / MFMA_F32_PEAK, 4)},
    }
    if not args.no_cpu and args.cpu_seconds > 0:
        from threadpoolctl import threadpool_limits

        from oracle import pgd_oracle as P
        Hc = w.H.astype(np.complex128)
        lam, eta = [1.0 / 15.0] * I, [1.0 / L] * I
        n = 0
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            while time.perf_counter() - t0 < min(args.cpu_seconds, 5.0):
                P.unfolded(Hc[n % B:n % B + 250], g, 1.0, lam, eta)
                n += 250
            el = time.perf_counter() - t0
        res["cpu_oracle"] = {"ufpgd20_ms_per_5000": round(el / n * B * 1e3, 2), "cores": 1,
                             "kind": "oracle", "sample": f"{n} channels in {el:.1f} s"}
    return res


def pa_phase(w, D, WL, torch, params, ap0, gpts):
    """The PA-consumption-aware precoder (eq. optim1 by normalised PGD, lambda =
    1/15, 5000 iterations) on the benchmark room: the step's K = 8 users, SINR
    targets 10 dB, noise -90 dBm.  Reports its PCG against ZF with the same
    targets, the APs it switches off and the SINR range; times the precoder
    and the 512 x 512 power + SINR map of the sparse W; then the precoder's
    throughput over 1024 user draws in the same room (one launch)."""
    import numpy as np

    K, M, N = w.K, w.M, w.grid.n
    gamma = np.full(K, 10.0)
    it = 5000
    lam = torch.full((it,), 1.0 / 15.0, dtype=torch.float64, device="cuda")
    er = torch.ones((it,), dtype=torch.float64, device="cuda")

    def timed(fn, reps):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ap = torch.from_numpy(w.ap_xyz).cuda()                  # [1][M][3]
    users = torch.from_numpy(w.user_xyz).cuda()             # [1][K][3]
    H = D.channel(params, ap, D.list_points(users, K), prec="f32")
    r = D.pa_precoder(H, lam, er, gamma, w.sigma2)
    ms_pa = timed(lambda: D.pa_precoder(H, lam, er, gamma, w.sigma2, out=r), 3)
    zf = D.beamform(H, "zf", gamma, w.sigma2, 0.0, "f32")
    mp = D.MapResult(torch.empty(N, device="cuda"), torch.empty(N, device="cuda"),
                     torch.empty(N, dtype=torch.int32, device="cuda"), None)
    Wpa = r.W[0].contiguous()
    ms_map = timed(lambda: D.powermap(params, ap0, Wpa, gpts, w.sigma2, "f32", out=mp), 20)
    mz = D.powermap(params, ap0, zf.W[0].contiguous(), gpts, w.sigma2, "f32")
    sinr_db = 10 * torch.log10(r.sinr[0])
    ratio_db = 10 * torch.log10(mp.power.double() / mz.power.double())

    B = 1024
    rng = np.random.default_rng(11)
    ub = torch.from_numpy(np.stack([WL.uniform_positions(rng, K, 20.0, 20.0, 1.2)
                                    for _ in range(B)])).cuda()
    apb = ap.expand(B, M, 3).contiguous()
    Hb = D.channel(params, apb, D.list_points(ub, K), prec="f32")
    rb = D.pa_precoder(Hb, lam, er, gamma, w.sigma2)
    ms_b = timed(lambda: D.pa_precoder(Hb, lam, er, gamma, w.sigma2, out=rb), 1)
    zfb = D.beamform(Hb, "zf", gamma, w.sigma2, 0.0, "f32")
    pcg_b = (zfb.l21 / rb.l21)
    off_b = (rb.p_ant == 0).sum(dim=1).double()
    flops = 16 * K * K * M * it
    hall = pa_hall(D, WL, torch, lam, er, timed)
    return {
        "workload": f"room deployment: M={M} jittered ceiling APs, the step's K={K} users, "
                    "SINR targets 10 dB, noise -90 dBm; lambda 1/15, eta = 1/lambda_max, "
                    f"{it} iterations",
        "precoder_ms": round(ms_pa, 3),
        "pcg_vs_zf": round((zf.l21[0] / r.l21[0]).item(), 4),
        "aps_off": int((r.p_ant[0] == 0).sum().item()),
        "sinr_db_min": round(sinr_db.min().item(), 3),
        "sinr_db_max": round(sinr_db.max().item(), 3),
        "map_ms": round(ms_map, 4),
        "map_power_vs_zf_db": {"median": round(ratio_db.median().item(), 3),
                               "p5": round(ratio_db.quantile(0.05).item(), 3),
                               "p95": round(ratio_db.quantile(0.95).item(), 3)},
        "batched": {"deployments": B, "ms": round(ms_b, 3),
                    "deployments_per_s": round(B / (ms_b * 1e-3), 1),
                    "tflops": round(flops * B / (ms_b * 1e-3) / 1e12, 2),
                    "mean_pcg": round(pcg_b.mean().item(), 4),
                    "min_pcg": round(pcg_b.min().item(), 4),
                    "mean_aps_off": round(off_b.mean().item(), 2)},
        "hall": hall,
        "serving": pa_serving(w, D, WL, torch),
    }


def pa_serving(w, D, WL, torch, rate=500.0, seconds=2.0):
    """Precoder-design queries in the serving runtime: a Poisson stream (rate
    1/s, `seconds` long) into one server holding the benchmark room; half the
    queries are DMIMO_PA (20-layer PGD schedule, lambda 1/15, targets 10 dB),
    half ZF; each brings 8 fresh users and asks for a 256 x 256 power + SINR
    map at 1.2 m.  Latency = completion - arrival, per kind."""
    import numpy as np

    rng = np.random.default_rng(12)
    n = int(rate * seconds)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, n))
    kinds = np.where(rng.random(n) < 0.5, "pa", "zf")
    users = [WL.uniform_positions(rng, w.K, 20.0, 20.0, 1.2) for _ in range(n)]
    side = 256
    grid = WL.Grid(0.0, 0.0, 20.0 / side, 20.0 / side, 1.2, side, side)
    pts = D.grid_points(grid)
    bufs = [(torch.empty(side * side, device="cuda"), torch.empty(side * side, device="cuda"))
            for _ in range(128)]
    free = list(range(len(bufs)))
    srv = D.Server(4 << 30, 64)
    dep = srv.add_deployment(D.channel_params(w.freq_hz), w.ap_xyz[0])
    srv.set_pa_schedule([1.0 / 15.0] * 20, [1.0] * 20, 10.0)
    torch.cuda.synchronize()
    outstanding, lat = [], {"pa": [], "zf": []}
    t0 = time.monotonic() + 0.05

    def reap():
        keep = []
        for tk, kind, bi, ta in outstanding:
            st, _, td = srv.poll(tk)
            if st >= D.Q_DONE:
                lat[kind].append(td - ta)
                srv.release(tk)
                free.append(bi)
            else:
                keep.append((tk, kind, bi, ta))
        outstanding[:] = keep

    for i in range(n):
        ta = t0 + arrivals[i]
        while time.monotonic() < ta or not free:
            if outstanding:
                reap()
        bi = free.pop()
        tk = srv.submit(dep, users[i], kinds[i], pts, w.sigma2, w.p_total, "f32", bufs[bi][0],
                        bufs[bi][1])
        outstanding.append((tk, kinds[i], bi, ta))
    while outstanding:
        srv.wait(outstanding[0][0], 30.0)
        reap()
    srv.close()
    out = {"workload": f"Poisson {rate:.0f} q/s for {seconds:.0f} s into one server holding the "
                       f"room: half PA-aware precoder queries (20 PGD layers), half ZF; 8 users "
                       f"and a {side} x {side} power + SINR map each"}
    for kind, v in lat.items():
        a = np.array(v) * 1e3
        out[kind] = {"queries": len(a), "p50_ms": round(float(np.percentile(a, 50)), 3),
                     "p99_ms": round(float(np.percentile(a, 99)), 3)}
    return out


def pa_hall(D, WL, torch, lam, er, timed):
    """The PA-aware precoder on the hall (32 users, 32 x 32 ceiling APs, 5.8
    GHz, targets 10 dB, -90 dBm) on the slab path, and the full 2048 x 2048
    power + SINR map of its sparse W."""
    import numpy as np

    w = WL.hall_workload()
    K, M, N = w.K, w.M, w.grid.n
    gamma = np.full(K, 10.0)
    params = D.channel_params(w.freq_hz)
    ap = torch.from_numpy(w.ap_xyz).cuda()
    H = D.channel(params, ap, D.list_points(torch.from_numpy(w.user_xyz).cuda(), K), prec="f32")
    r = D.pa_precoder(H, lam, er, gamma, w.sigma2)
    ms = timed(lambda: D.pa_precoder(H, lam, er, gamma, w.sigma2, out=r), 2)
    zf = D.beamform(H, "zf", gamma, w.sigma2, 0.0, "f32")
    gpts = D.grid_points(w.grid)
    ap0 = ap[0].contiguous()
    mp = D.powermap(params, ap0, r.W[0].contiguous(), gpts, w.sigma2, "f32", want_best=False)
    ms_map = timed(lambda: D.powermap(params, ap0, r.W[0].contiguous(), gpts, w.sigma2, "f32",
                                      out=mp), 2)
    sinr_db = 10 * torch.log10(r.sinr[0])
    return {"workload": f"hall: M={M} regular ceiling APs (50 x 50 m, z = 5 m), K={K} users, "
                        f"5.8 GHz, targets 10 dB, noise -90 dBm; {lam.numel()} iterations",
            "precoder_ms": round(ms, 3),
            "pcg_vs_zf": round((zf.l21[0] / r.l21[0]).item(), 4),
            "aps_off": int((r.p_ant[0] == 0).sum().item()),
            "sinr_db_min": round(sinr_db.min().item(), 3),
            "sinr_db_max": round(sinr_db.max().item(), 3),
            "map_2048x2048_ms": round(ms_map, 3),
            "map_terms": N * M}


def cpu_baseline(w, bf, maps, budget_s):
    """Oracle timed on a bounded sample of the step, single-threaded.

    The sample is the user-side calls (channel, MR and ZF precoders with
    their SINR and L2,1 epilogues) plus power and SINR maps of both precoders
    on 16 random grid rows, repeated until the budget is spent.

    Also reports the dB error of the GPU chain (GPU H -> GPU W -> GPU map)
    against the oracle chain (oracle H -> oracle W -> oracle map) on the first
    sampled rows.  No GPU output enters the oracle.
    """
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import dberror
    from oracle import dmimo_oracle as O

    g = w.grid
    nx = g.nx
    rows_per_rep = 16
    pts_all = O.grid_points(g.x0, g.y0, g.dx, g.dy, g.z, g.nx, g.ny)
    aps = w.ap_xyz[0]
    K, M = w.K, w.M
    gpu = {p: (maps[p].power.cpu().numpy(), maps[p].sinr.cpu().numpy()) for p in maps}
    pairs = {"power": [], "sinr": []}
    terms = 0
    reps = 0
    rng = np.random.default_rng(0)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget_s:
            Hu = O.los_channel(w.user_xyz[0], aps, w.freq_hz)
            Wmr = O.mr_precoder(Hu, w.p_total)
            Wzf, _ = O.zf_precoder(Hu, None, w.sigma2, w.p_total)
            for Wp in (Wmr, Wzf):
                O.user_sinr(Hu, Wp, w.sigma2)
                O.antenna_power(Wp)
                O.l21_norm(Wp)
            terms += 3 * K * M
            j0 = int(rng.integers(0, g.ny - rows_per_rep + 1))
            sl = slice(j0 * nx, (j0 + rows_per_rep) * nx)
            Hg = O.los_channel(pts_all[sl], aps, w.freq_hz)
            for name, Wp in (("mr", Wmr), ("zf", Wzf)):
                y = O.power_map(Hg, Wp)
                s, _ = O.sinr_map(Hg, Wp, w.sigma2)
                terms += (sl.stop - sl.start) * M
                if reps < 8:
                    pairs["power"].append((gpu[name][0][sl], y))
                    pairs["sinr"].append((gpu[name][1][sl], s))
            reps += 1
        elapsed = time.perf_counter() - t0
    err = {}
    for k, pr in pairs.items():
        y = np.concatenate([p[0] for p in pr])
        r = np.concatenate([p[1] for p in pr])
        sm = dberror.summary(y, r, 0.01)
        err[k] = {"max_db": sm["max_db"], "p99_db": sm["p99_db"], "n": sm["n"],
                  "n_below_floor": sm["n_below_floor"], "n_over_0.01dB": sm["n_fail"]}
    err["compared"] = "GPU chain vs oracle chain (users -> precoder -> map), both precoders"
    cpu = {
        "value": round(terms / elapsed / 1e9, 6),
        "unit": "G h/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{reps} reps of the step's user-side calls plus power+SINR maps of MR and ZF "
                  f"on {rows_per_rep} random grid rows ({rows_per_rep * nx} points each): "
                  f"{terms} terms in {elapsed:.1f} s",
    }
    return cpu, err


if __name__ == "__main__":
    main()
