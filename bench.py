#!/usr/bin/env python3
"""Benchmark of the distributed-MIMO hot path on one MI355X.

Headline workload ("hall", the largest single-GPU configuration): M = 1024
APs on a regular 32x32 ceiling grid (pitch 1.5625 m, z = 5 m) of a 50x50x5 m
hall, 5.8 GHz, K = 32 users at z = 1 m, ZF at 1 W, noise -90 dBm, power + SINR
map on a 2048x2048 grid at z = 1 m.  One step is one pass of the whole path,
with inputs already resident in HBM:

  1. dmimo_beamform_users  the users' LoS channels H (K x M) and their ZF
                           precoder at 1 W with p_m, L2,1, SINR_k and R_sum
                           (channel kernel, then the wide ZF path: per-tile
                           Gram shares, FP64 Gauss-Jordan inverse, W)
  2. dmimo_powermap        power + SINR + best-stream map over the 2048^2 grid,
                           the channel synthesised in the kernel (FP64
                           distance and phase) and contracted with W

The headline precision is the configuration's: FP16 hi/lo split products on
the matrix cores with FP32 accumulation (``f16x3``).  The same step in plain
FP32 and in BF16x3 is timed beside it (``fp32``, ``bf16x3``), with the
speed-up of the mixed path.

value = channel terms h[n,m] synthesised and consumed per second over the
whole step (K M for the channels, K M for the precoder, N M for the map), in
G h/s.

The JSON line also carries:
* ``roofline`` for the dominant kernel (the map).  Its launch duration is the
  mean of a dedicated pass of HIP-event pairs on the launching stream (at
  least 20 launches).  The kernel is bound by its VALU work (synthesis and
  hi/lo split); the matrix-core fraction is reported beside it.
* ``err_db``: every result of the GPU chain against the FP64 oracle chain
  (oracle users -> oracle ZF -> oracle map) in dB, for each precision: the
  map on sampled grid rows, and the per-user SINR_k.
* ``cpu_baseline``: the FP64 oracle timed on the host's cores (all of them,
  one process per core, and one core alone) on a bounded sample of the same
  step: the users' channel and ZF plus map rows.
* Secondary configurations: ``room`` (the 512x512 MR + ZF room step),
  ``focus`` (the FP64 MR focusing map), ``batched`` (Rician Gram + ZF over
  many deployments), ``paper`` (the paper's ZF sum rate), ``serving``
  (Poisson queries, p50/p99, FP16x3 maps with the same stream in FP32 beside
  them; ``serving_sweep``: p50/p99 at 500 to 4000 queries/s), ``pgd`` and
  ``pa`` (the paper's solver), and
  ``channel`` (the channel materialised in HBM), each with its dB errors.

Only the CPU-baseline and error legs import the oracle; they run before the
first GPU call (the oracle values) and after the timed regions.
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
# roofline model of the power-map kernels (VALU issue slots)
# ---------------------------------------------------------------------------
# MI355X: 256 CUs x 4 SIMDs x 16 lanes per clock x 2.4 GHz = 39.3e12 lane-slots/s.
# FP64 add/mul/FMA, conversions and unpacked FP32 ops issue at that rate; the
# transcendentals (rsq, sin, cos) at half of it (2 slots, measured).
VALU_PEAK_SLOTS = 256 * 4 * 16 * 2.4e9
# Algorithmic slots per term for FP64 distance/phase + FP32 synthesis of a
# point in general position:
#   d^2: 3 sub + mul + 2 FMA                                      6
#   d = sqrt(d^2): cvt, rsq (2), cvt, 2 mul, 2 FMA (one Newton)   8
#   phase: fract, cvt                                             2
#   sin (2) + cos (2)                                             4
#   amplitude and h = amp (cos, -sin): 3 mul                      3
# = 23 slots.  The split-precision maps add the hi/lo split of h: two
# packed conversions and two mixed-precision residuals per term, 4 slots.
# The K-stream contraction runs on the matrix cores (FP32, or FP16/BF16 x3).
SYNTH_SLOTS = 23
SPLIT_SLOTS = 4
MFMA_F32_PEAK = 157.3e12
MFMA_F16_PEAK = 2.5e15
HBM_PEAK = 8.0e12   # MI355X HBM3E, bytes/s


def alg_slots_per_term(K: int, prec: str = "f32") -> int:
    if prec in ("f16x3", "bf16x3"):
        return SYNTH_SLOTS + SPLIT_SLOTS
    # FP32: K <= 2 maps run the contraction on the VALU (4K FMA per term)
    return SYNTH_SLOTS if K >= 3 else SYNTH_SLOTS + 4 * K


def mfma_flops_per_term(K: int, prec: str) -> int:
    # 8K real flops per term (K complex MACs); the split products run three
    return 8 * K * (3 if prec in ("f16x3", "bf16x3") else 1)


def _src_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


# every file the map kernels are compiled from (a traffic summary is only
# valid for these exact sources)
POWERMAP_SOURCES = ["paper_2304_12745_amd/csrc/powermap.hip",
                    "paper_2304_12745_amd/csrc/powermap_mfma.hip",
                    "paper_2304_12745_amd/csrc/powermap_mfma.h",
                    "paper_2304_12745_amd/csrc/powermap_body.h",
                    "paper_2304_12745_amd/csrc/powermap_common.h",
                    "paper_2304_12745_amd/csrc/split16.h",
                    "paper_2304_12745_amd/csrc/kernels.h",
                    "paper_2304_12745_amd/csrc/dmimo_internal.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "powermap_hall_traffic.json")
ROOM_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "powermap_room_traffic.json")
ROOM_F16_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "powermap_room_f16x3_traffic.json")


def load_traffic(kernel_hash: str, path: str = None):
    """HBM bytes per launch from a committed rocprofv3 --pmc summary.

    None if there is none, or if it was taken on other kernel sources.
    """
    try:
        with open(path or TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != kernel_hash:
        return None
    return t.get("bytes_per_launch")


def host_info():
    """Host CPU model and core count (where the oracle baseline runs)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": usable, "os_cpu_count": os.cpu_count()}


def parse_args():
    p = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=50)
    p.add_argument("--warmup", type=int, default=10)
    p.add_argument("--ramp-seconds", type=float, default=0.3,
                   help="untimed map launches before the first warm-up step (brings the GPU "
                        "clocks up; not counted as warm-up steps)")
    p.add_argument("--event-launches", type=int, default=30,
                   help="map launches in the dedicated HIP-event pass of the roofline (>= 20)")
    p.add_argument("--cpu-seconds", type=float, default=10.0,
                   help="wall budget of the all-core oracle baseline (the one-core leg takes "
                        "half of it); 0 disables both")
    p.add_argument("--cpu-workers", type=int, default=16,
                   help="at most this many oracle processes (the GPU box's CPU share is 16)")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--serve-seconds", type=float, default=30.0,
                   help="measured window of the serving phase (0 disables it)")
    p.add_argument("--serve-warmup", type=float, default=5.0)
    p.add_argument("--serve-rate", type=float, default=2000.0, help="Poisson arrival rate (1/s)")
    p.add_argument("--serve-prec", default="f16x3", choices=["f32", "f16x3", "bf16x3"],
                   help="precision of the served maps (the FP32 stream is also run, shorter, "
                        "as the comparison; --serve-compare-seconds 0 skips it)")
    p.add_argument("--serve-compare-seconds", type=float, default=10.0)
    p.add_argument("--no-serve-sweep", dest="serve_sweep", action="store_false",
                   help="skip the load sweep (by default, when the stream is served, it is "
                        "also served at 500, 1000, 2000 and 4000 queries/s, 3 s each after 1 s)")
    p.add_argument("--room-steps", type=int, default=500)
    p.add_argument("--room-warmup", type=int, default=2000)
    p.add_argument("--room-streams", type=int, default=2)
    p.add_argument("--event-every", type=int, default=10,
                   help="room step: record the map event pair on every n-th timed step")
    p.add_argument("--nx", type=int, default=512, help="room grid side")
    p.add_argument("--no-room", action="store_true")
    p.add_argument("--no-twins", action="store_true", help="skip the FP32 and BF16x3 hall steps")
    p.add_argument("--no-pgd", action="store_true", help="skip the PGD / unfolded-PGD phase")
    p.add_argument("--no-pa", action="store_true", help="skip the PA-aware precoder phase")
    p.add_argument("--no-channel", action="store_true",
                   help="skip the materialised-channel bandwidth phase")
    p.add_argument("--no-batched", action="store_true",
                   help="skip the batched Gram + ZF phase")
    p.add_argument("--only-hall", action="store_true",
                   help="the hall steps and their roofline only (profiling runs)")
    p.add_argument("--only-batched", action="store_true",
                   help="the batched phase only, printed as its own JSON line (profiling runs)")
    return p.parse_args()


# ---------------------------------------------------------------------------
# oracle legs (CPU; imported only here)
# ---------------------------------------------------------------------------

HALL_ERR_ROWS = (0, 301, 602, 1023, 1024, 1445, 1746, 2047)


def _hall_oracle_rows(rows):
    """Oracle chain of the hall step for the given grid rows: the users'
    channel and ZF at 1 W, then power and SINR maps on those rows.  Returns
    (terms, power [rows][nx], sinr [rows][nx], user SINR [K])."""
    import numpy as np
    from oracle import dmimo_oracle as O
    from paper_2304_12745_amd import workloads as WL
    w = WL.hall_workload()
    g = w.grid
    aps = w.ap_xyz[0]
    Hu = O.los_channel(w.user_xyz[0], aps, w.freq_hz)
    Wz, _ = O.zf_precoder(Hu, None, w.sigma2, w.p_total)
    su = O.user_sinr(Hu, Wz, w.sigma2)
    O.antenna_power(Wz)
    O.l21_norm(Wz)
    terms = 2 * w.K * w.M
    pw, sn = [], []
    xs = g.x0 + (np.arange(g.nx) + 0.5) * g.dx
    for j in rows:
        y = g.y0 + (j + 0.5) * g.dy
        pts = np.stack([xs, np.full(g.nx, y), np.full(g.nx, g.z)], axis=1)
        Hg = O.los_channel(pts, aps, w.freq_hz)
        pw.append(O.power_map(Hg, Wz))
        sn.append(O.sinr_map(Hg, Wz, w.sigma2)[0])
        terms += g.nx * w.M
    return terms, np.array(pw), np.array(sn), su


def _oracle_worker(args):
    """One oracle process: rows start, start + stride, ... until the deadline
    (wall clock).  One numpy/BLAS thread."""
    start, stride, deadline = args
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        terms, n, j = 0, 0, start
        while time.time() < deadline or n == 0:
            t, _, _, _ = _hall_oracle_rows([j % 2048])
            terms += t
            n += 1
            j += stride
    return terms, n


def cpu_baseline_hall(budget_s: float, max_workers: int):
    """The FP64 oracle on the hall step, timed on all host cores (one process
    each, rows dealt round-robin) and on one core, before any GPU call.  Also
    returns the oracle values that the error report compares with."""
    import multiprocessing as mp

    from threadpoolctl import threadpool_limits

    info = host_info()
    # the error rows first (one core, untimed)
    with threadpool_limits(limits=1):
        _, ref_p, ref_s, ref_u = _hall_oracle_rows(HALL_ERR_ROWS)
    ref = {"power": ref_p, "sinr": ref_s, "user_sinr": ref_u}
    if budget_s <= 0:
        return None, ref
    workers = max(1, min(max_workers, info["nproc"] or 1))
    ctx = mp.get_context("fork")       # no GPU has been touched in this process yet
    t0 = time.time()
    deadline = t0 + budget_s
    with ctx.Pool(workers) as pool:
        res = pool.map(_oracle_worker, [(i * 7, workers * 7 + 1, deadline) for i in range(workers)])
    el_all = time.time() - t0
    terms_all = sum(r[0] for r in res)
    rows_all = sum(r[1] for r in res)
    # one core
    one_budget = budget_s / 2
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        terms1, n1, j = 0, 0, 3
        while time.perf_counter() - t0 < one_budget or n1 == 0:
            t, _, _, _ = _hall_oracle_rows([j % 2048])
            terms1 += t
            n1 += 1
            j += 97
        el1 = time.perf_counter() - t0
    full = 2 * 32 * 1024 + 2048 * 2048 * 1024
    v_all = terms_all / el_all / 1e9
    v1 = terms1 / el1 / 1e9
    cpu = {
        "value": round(v_all, 6),
        "unit": "G h/s",
        "cores": workers,
        "kind": "oracle",
        "sample": (f"hall step, oracle chain (users' channel + ZF + power and SINR map rows), "
                   f"{rows_all} grid rows of 2048 points x 1024 APs x 32 streams on {workers} "
                   f"processes (one BLAS thread each) in {el_all:.1f} s; work per row is "
                   f"uniform, so the rate extrapolates linearly to the full map: "
                   f"{full / (v_all * 1e9):.0f} s per step"),
        "one_core": {"value": round(v1, 6), "unit": "G h/s",
                     "sample": f"{n1} grid rows in {el1:.1f} s"},
        "host": info,
    }
    return cpu, ref


def db_report(y, ref, tol, floor_rel=1e-6):
    from oracle import dberror
    s = dberror.summary(y, ref, tol, floor_rel)
    return {"max_db": s["max_db"], "p99_db": s["p99_db"], "n": s["n"],
            "n_below_floor": s["n_below_floor"], f"n_over_{tol}dB": s["n_fail"]}


def plain_db(y, ref):
    import numpy as np
    e = np.abs(10.0 * np.log10(np.asarray(y, np.float64) / np.asarray(ref, np.float64))).ravel()
    return {"max_db": float(e.max()), "p99_db": float(np.percentile(e, 99)), "n": int(e.size)}


# ---------------------------------------------------------------------------
# the hall step
# ---------------------------------------------------------------------------

class HallStep:
    """The hall step at one precision, with its outputs preallocated."""

    def __init__(self, D, WL, torch, prec):
        self.D, self.torch, self.prec = D, torch, prec
        w = self.w = WL.hall_workload()
        self.K, self.M, self.N = w.K, w.M, w.grid.n
        self.params = D.channel_params(w.freq_hz)
        self.ap = torch.from_numpy(w.ap_xyz).cuda()            # [1][M][3]
        self.ap0 = self.ap[0].contiguous()
        self.users = torch.from_numpy(w.user_xyz).cuda()      # [1][K][3]
        self.gpts = D.grid_points(w.grid)
        self.pre = D.beamform_users(self.params, self.ap, self.users, ("zf",), None, w.sigma2,
                                    w.p_total, prec)
        self.W = self.pre.W[0, 0]                              # [K][M], contiguous
        N = self.N
        self.maps = D.MapResult(torch.empty(N, device="cuda"), torch.empty(N, device="cuda"),
                                torch.empty(N, dtype=torch.int32, device="cuda"), None)
        self.terms = 2 * self.K * self.M + N * self.M

    def precoder(self):
        w = self.w
        self.D.beamform_users(self.params, self.ap, self.users, ("zf",), None, w.sigma2,
                              w.p_total, self.prec, out=self.pre)

    def map(self):
        self.D.powermap(self.params, self.ap0, self.W, self.gpts, self.w.sigma2, self.prec,
                        out=self.maps)

    def step(self):
        self.precoder()
        self.map()

    def timed(self, warmup, steps):
        torch = self.torch
        for _ in range(warmup):
            self.step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            self.step()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps

    def map_events(self, launches):
        """Mean duration of the map launch: one HIP-event pair around each of
        `launches` back-to-back launches on the launching stream (torch's
        current stream, which the binding passes to the library)."""
        torch = self.torch
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * launches)]
        self.map()
        torch.cuda.synchronize()
        for i in range(launches):
            ev[2 * i].record()
            self.map()
            ev[2 * i + 1].record()
        torch.cuda.synchronize()
        ts = sorted(ev[2 * i].elapsed_time(ev[2 * i + 1]) for i in range(launches))
        return sum(ts) / launches, ts[0], ts[len(ts) // 2]

    def ramp(self, seconds):
        torch = self.torch
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < seconds:
            for _ in range(10):
                self.map()
            torch.cuda.synchronize()

    def sampled(self):
        """Map rows HALL_ERR_ROWS and the users' SINR, on the host."""
        import numpy as np
        torch = self.torch
        torch.cuda.synchronize()
        nx = self.w.grid.nx
        p = self.maps.power.view(-1, nx)[list(HALL_ERR_ROWS)].double().cpu().numpy()
        s = self.maps.sinr.view(-1, nx)[list(HALL_ERR_ROWS)].double().cpu().numpy()
        u = self.pre.sinr[0, 0].cpu().numpy()
        return {"power": p, "sinr": s, "user_sinr": np.asarray(u), "info": int(self.pre.info[0, 0])}


def hall_phase(args, D, WL, torch):
    """The headline (FP16x3) and its FP32 and BF16x3 twins."""
    out = {}
    head = HallStep(D, WL, torch, "f16x3")
    head.ramp(args.ramp_seconds)
    ms = head.timed(args.warmup, args.steps)
    launch, lmin, lmed = head.map_events(max(20, args.event_launches))
    out["f16x3"] = {"ms_per_step": ms, "map_launch_ms": launch, "map_launch_min_ms": lmin,
                    "map_launch_median_ms": lmed, "sample": head.sampled(), "step": head}
    if not args.no_twins:
        for prec in ("f32", "bf16x3"):
            tw = HallStep(D, WL, torch, prec)
            ms = tw.timed(args.warmup, args.steps)
            launch, lmin, lmed = tw.map_events(max(20, args.event_launches))
            out[prec] = {"ms_per_step": ms, "map_launch_ms": launch, "map_launch_min_ms": lmin,
                         "map_launch_median_ms": lmed, "sample": tw.sampled()}
            del tw
            torch.cuda.empty_cache()
    return out


def hall_roofline(K, N, M, prec, launch_ms, khash, traffic):
    terms = N * M
    slots = alg_slots_per_term(K, prec)
    achieved = slots * terms / (launch_ms * 1e-3) / 1e12
    peak = VALU_PEAK_SLOTS / 1e12
    mf = mfma_flops_per_term(K, prec) * terms
    mpeak = MFMA_F16_PEAK if prec in ("f16x3", "bf16x3") else MFMA_F32_PEAK
    t_valu = slots * terms / VALU_PEAK_SLOTS
    t_mfma = mf / mpeak
    kern = {"f16x3": "powermap_x3w_kernel<4, 2, false, 8>",
            "bf16x3": "powermap_x3w_kernel<4, 2, true, 8>",
            "f32": "powermap_mfma_kernel<4, 2, 8>"}[prec]
    return {
        "bound": "alu",
        "kernel": f"{kern}, the 2048 x 2048 hall map (K = 32, M = 1024)",
        "achieved": round(achieved, 3),
        "peak": round(peak, 3),
        "unit": "T VALU lane-slots/s",
        "frac": round(achieved / peak, 4),
        "traffic": traffic,
        "launch_ms": round(launch_ms, 5),
        "alg_slots_per_term": slots,
        "terms_per_launch": terms,
        "mfma": {"achieved": round(mf / (launch_ms * 1e-3) / 1e12, 3),
                 "peak": round(mpeak / 1e12, 1), "unit": "TFLOP/s",
                 "frac": round(mf / (launch_ms * 1e-3) / mpeak, 4),
                 "flops_per_term": mfma_flops_per_term(K, prec)},
        # the FP16/BF16 matrix cores overlap the VALU (the floor is the larger
        # of the two times); FP32 MFMA does not (the floor is their sum)
        "floor_ms": round((max(t_valu, t_mfma) if prec != "f32" else t_valu + t_mfma) * 1e3, 4),
        "frac_of_floor": round((max(t_valu, t_mfma) if prec != "f32" else t_valu + t_mfma) * 1e3
                               / launch_ms, 4),
        "source_hash": khash,
    }


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

    # counting devices does not initialise the GPU, so the oracle processes
    # below can still be forked from this one
    if torch.cuda.device_count() < 1:
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)

    from paper_2304_12745_amd import dmimo as D
    from paper_2304_12745_amd import workloads as WL

    cpu, ref = None, None
    if not args.no_cpu:
        cpu, ref = cpu_baseline_hall(args.cpu_seconds, args.cpu_workers)

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    D.lib()
    torch.cuda.set_device(0)

    # a plain copy of known size, for scaling the HBM counters of a profiled run
    cp_src = torch.empty(64 << 20, dtype=torch.uint8, device="cuda")
    cp_dst = torch.empty_like(cp_src)
    cp_dst.copy_(cp_src)

    if args.only_batched:
        print(json.dumps({"batched": batched_phase(D, WL, torch, args.event_launches)}), flush=True)
        return

    hall = hall_phase(args, D, WL, torch)
    head = hall["f16x3"]
    hs = head.pop("step")
    K, M, N = hs.K, hs.M, hs.N
    terms = hs.terms
    value = terms / (head["ms_per_step"] * 1e-3) / 1e9
    khash = _src_hash(POWERMAP_SOURCES)
    traffic = load_traffic(khash)

    out = {
        "metric": "channel-term evals/sec (G h[n,m]/s) + p99 query latency, mixed vs FP32",
        "value": round(value, 3),
        "unit": "G h/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16x3",
        "data": "synthetic",
        "config": {
            "workload": "hall: M=1024 APs on a regular 32x32 ceiling grid (pitch 1.5625 m, z=5 m) "
                        "of a 50x50x5 m hall, 5.8 GHz, K=32 users at z=1 m, ZF at 1 W, noise "
                        "-90 dBm, 2048x2048 power+SINR map at z=1 m; FP64 distance/phase, FP32 "
                        "synthesis, FP16 hi/lo x3 MFMA contraction with FP32 accumulation",
            "M": M, "K": K, "N": N, "terms_per_step": terms,
            "step": "dmimo_beamform_users (users' LoS channels + ZF, wide path) + dmimo_powermap",
        },
        "roofline": hall_roofline(K, N, M, "f16x3", head["map_launch_ms"], khash, traffic),
    }
    out["roofline"]["event_samples"] = max(20, args.event_launches)
    out["roofline"]["launch_min_ms"] = round(head["map_launch_min_ms"], 5)
    out["roofline"]["launch_median_ms"] = round(head["map_launch_median_ms"], 5)

    # the twins: the same step in FP32 and in BF16x3
    for prec in ("f32", "bf16x3"):
        if prec not in hall:
            continue
        h = hall[prec]
        out["fp32" if prec == "f32" else prec] = {
            "ms_per_step": round(h["ms_per_step"], 5),
            "value": round(terms / (h["ms_per_step"] * 1e-3) / 1e9, 3),
            "map_launch_ms": round(h["map_launch_ms"], 5),
            "roofline": hall_roofline(K, N, M, prec, h["map_launch_ms"], khash, None),
        }
    if "f32" in hall:
        out["mixed_vs_fp32"] = {
            "speedup_step": round(hall["f32"]["ms_per_step"] / head["ms_per_step"], 3),
            "speedup_map_launch": round(hall["f32"]["map_launch_ms"] / head["map_launch_ms"], 3)}

    # every result of the GPU chain against the oracle chain, per precision
    if ref is not None:
        err = {}
        tol = {"f16x3": 0.1, "bf16x3": 0.1, "f32": 0.01}
        for prec in ("f16x3", "f32", "bf16x3"):
            if prec not in hall:
                continue
            smp = hall[prec]["sample"]
            err[prec] = {"power": db_report(smp["power"], ref["power"], tol[prec]),
                         "sinr": db_report(smp["sinr"], ref["sinr"], tol[prec]),
                         "user_sinr": plain_db(smp["user_sinr"], ref["user_sinr"]),
                         "zf_info": smp["info"]}
        err["compared"] = (f"GPU chain (users' channel -> ZF -> map) vs the FP64 oracle chain, "
                           f"grid rows {list(HALL_ERR_ROWS)} ({len(HALL_ERR_ROWS) * 2048} points) "
                           f"and the 32 users' SINR_k; tolerance 0.1 dB mixed, 0.01 dB FP32, "
                           f"floor rule at -60 dB below the sample's peak")
        out["err_db"] = err
    for prec in hall:
        hall[prec].pop("sample", None)
    del hs
    torch.cuda.empty_cache()

    if not args.only_hall:
        if not args.no_room:
            out["room"] = room_phase(args, D, WL, torch)
        out["focus"] = focus_phase(D, WL, torch)
        out["paper"] = paper_phase(D, WL, torch)
        if not args.no_channel:
            out["channel"] = channel_phase(D, WL, torch)
        if not args.no_batched:
            out["batched"] = batched_phase(D, WL, torch, args.event_launches)
        if args.serve_seconds > 0:
            out["serving"] = serving_phase(args, D, WL, torch)
            out["p99_query_ms"] = out["serving"]["p99_ms"]
            if args.serve_prec != "f32" and args.serve_compare_seconds > 0:
                # the same Poisson stream served in FP32 (shorter window)
                a2 = argparse.Namespace(**vars(args))
                a2.serve_prec, a2.serve_seconds, a2.serve_warmup = "f32", args.serve_compare_seconds, 2.0
                r = serving_phase(a2, D, WL, torch)
                out["serving"]["f32"] = {k: r[k] for k in ("measured_s", "queries", "failed", "p50_ms",
                                                           "p99_ms", "max_ms", "sustained_Gh_per_s")}
        if args.serve_seconds > 0 and args.serve_sweep:
            sweep = []
            for rate in (500.0, 1000.0, 2000.0, 4000.0):
                a2 = argparse.Namespace(**vars(args))
                a2.serve_rate, a2.serve_seconds, a2.serve_warmup = rate, 3.0, 1.0
                r = serving_phase(a2, D, WL, torch)
                sweep.append({k: r[k] for k in ("rate_qps", "queries", "p50_ms", "p99_ms", "max_ms",
                                                "sustained_Gh_per_s", "offered_Gh_per_s")})
            out["serving_sweep"] = sweep
        if not args.no_pgd:
            out["pgd"] = pgd_phase(args, D, WL, torch)
        if not args.no_pa:
            out["pa"] = pa_phase(WL.room_workload(nx=args.nx, ny=args.nx), D, WL, torch)
    if cpu is not None:
        out["cpu_baseline"] = cpu

    print(json.dumps(out), flush=True)


# ---------------------------------------------------------------------------
# secondary configurations
# ---------------------------------------------------------------------------

def room_phase(args, D, WL, torch):
    """The room step (M = 64, K = 8, MR + ZF, two 512x512 power + SINR +
    best-stream maps), FP32 and FP16x3, on one stream and on several; its map
    launch duration from HIP events; the GPU chain against the oracle chain on
    sampled rows."""
    w = WL.room_workload(nx=args.nx, ny=args.nx)
    K, M, N = w.K, w.M, w.grid.n
    params = D.channel_params(w.freq_hz)
    ap = torch.from_numpy(w.ap_xyz).cuda()
    ap0 = ap[0].contiguous()
    users = torch.from_numpy(w.user_xyz).cuda()
    gpts = D.grid_points(w.grid)
    H = torch.empty((1, K, M), dtype=torch.complex64, device="cuda")
    ra = argparse.Namespace(steps=args.room_steps, warmup=args.room_warmup,
                            event_every=args.event_every)
    ms_one, launch, maps, _ = run_steps(ra, "f32", w, D, params, ap, ap0, users, gpts, H)
    ms_n = run_steps(ra, "f32", w, D, params, ap, ap0, users, gpts, H,
                     nstreams=args.room_streams)[0] if args.room_streams > 1 else ms_one
    ms_mix, launch_mix, maps_mix, _ = run_steps(ra, "f16x3", w, D, params, ap, ap0, users, gpts, H)
    # distinct channel terms per step: the users' K M and the map's N M; the
    # map term feeds both precoders' streams in one contraction
    terms = K * M + N * M
    khash = _src_hash(POWERMAP_SOURCES)
    slots = alg_slots_per_term(2 * K)
    res = {
        "workload": f"room: M={M} APs jittered 8x8 ceiling grid 20x20x4 m, K={K} users, 3.5 GHz, "
                    f"MR+ZF at 1 W, noise -90 dBm, {w.grid.nx}x{w.grid.ny} power+SINR+best-stream "
                    "maps at z=1.2 m (both maps in one launch: one contraction of the 2K streams)",
        "terms_per_step": terms,
        "terms_counted": "distinct channel terms: K M of the users' channels + N M of the grid",
        "f32": {"ms_per_step_one_stream": round(ms_one, 5),
                "value_one_stream": round(terms / (ms_one * 1e-3) / 1e9, 3),
                "streams": args.room_streams, "ms_per_step": round(ms_n, 5),
                "value": round(terms / (ms_n * 1e-3) / 1e9, 3),
                "maps_launch_ms": round(launch, 5)},
        "f16x3": {"ms_per_step_one_stream": round(ms_mix, 5),
                  "value_one_stream": round(terms / (ms_mix * 1e-3) / 1e9, 3),
                  "maps_launch_ms": round(launch_mix, 5)},
        "roofline": {"bound": "alu",
                     "kernel": "powermap_mfma_kernel<2, 2, 8>: MR and ZF, 16 streams, one grid",
                     "alg_slots_per_term": slots,
                     "frac": round(slots * N * M / (launch * 1e-3) / VALU_PEAK_SLOTS, 4),
                     "mfma_f32_frac": round(8 * 2 * K * N * M / (launch * 1e-3) / MFMA_F32_PEAK, 4),
                     # FP32 MFMA does not co-issue with the VALU: the floor is
                     # the synthesis at the slot peak plus the contraction at
                     # the FP32 matrix-core peak
                     "floor_ms": round((slots * N * M / VALU_PEAK_SLOTS
                                        + 8 * 2 * K * N * M / MFMA_F32_PEAK) * 1e3, 5),
                     "frac_of_floor": round((slots * N * M / VALU_PEAK_SLOTS
                                             + 8 * 2 * K * N * M / MFMA_F32_PEAK) / (launch * 1e-3), 4),
                     "launch_ms": round(launch, 5),
                     "traffic": load_traffic(khash, ROOM_TRAFFIC_FILE), "source_hash": khash},
    }
    # the split FP16 contraction co-issues with the synthesis: its floor is
    # the larger of the VALU time and the FP16 matrix-core time
    sl16 = alg_slots_per_term(2 * K, "f16x3")
    t_v, t_m = sl16 * N * M / VALU_PEAK_SLOTS, mfma_flops_per_term(2 * K, "f16x3") * N * M / MFMA_F16_PEAK
    res["roofline_f16x3"] = {
        "bound": "alu",
        "kernel": "powermap_x3w_kernel<2, 2, false, 8>: MR and ZF, 16 streams, one grid, FP16 hi/lo x3",
        "alg_slots_per_term": sl16,
        "frac": round(sl16 * N * M / (launch_mix * 1e-3) / VALU_PEAK_SLOTS, 4),
        "mfma_f16_frac": round(t_m / (launch_mix * 1e-3), 4),
        "floor_ms": round(max(t_v, t_m) * 1e3, 5),
        "frac_of_floor": round(max(t_v, t_m) / (launch_mix * 1e-3), 4),
        "launch_ms": round(launch_mix, 5),
        "traffic": load_traffic(khash, ROOM_F16_TRAFFIC_FILE), "source_hash": khash}
    res["err_db"] = room_errors(w, maps, maps_mix)
    return res


def room_errors(w, maps, maps_mix, rows=(0, 1, 137, 255, 256, 511)):
    """The GPU maps of the room step (GPU H -> GPU W -> GPU map) against the
    oracle chain on sampled rows, FP32 and FP16x3."""
    import numpy as np
    from oracle import dmimo_oracle as O
    g = w.grid
    aps = w.ap_xyz[0]
    Hu = O.los_channel(w.user_xyz[0], aps, w.freq_hz)
    Wp = {"mr": O.mr_precoder(Hu, w.p_total), "zf": O.zf_precoder(Hu, None, w.sigma2, w.p_total)[0]}
    xs = g.x0 + (np.arange(g.nx) + 0.5) * g.dx
    pts = np.concatenate([np.stack([xs, np.full(g.nx, g.y0 + (j + 0.5) * g.dy),
                                    np.full(g.nx, g.z)], axis=1) for j in rows])
    Hg = O.los_channel(pts, aps, w.freq_hz)
    out = {}
    for tag, mp, tol in (("f32", maps, 0.01), ("f16x3", maps_mix, 0.1)):
        for p in ("mr", "zf"):
            pw = mp[p].power.view(g.ny, g.nx)[list(rows)].double().cpu().numpy().ravel()
            sn = mp[p].sinr.view(g.ny, g.nx)[list(rows)].double().cpu().numpy().ravel()
            out[f"{tag}_{p}"] = {"power": db_report(pw, O.power_map(Hg, Wp[p]), tol),
                                 "sinr": db_report(sn, O.sinr_map(Hg, Wp[p], w.sigma2)[0], tol)}
    out["compared"] = f"GPU chain vs oracle chain, grid rows {list(rows)}"
    return out


def focus_phase(D, WL, torch):
    """The FP64 MR focusing map (M = 16 APs, 920 MHz, 64x64 grid): the focal
    point's channel, MR at 1 W and the map, all in FP64; every point against
    the oracle, and the focal-point closed form y = P sum_m |h_m|^2."""
    import numpy as np
    from oracle import dmimo_oracle as O
    w = WL.focus_workload()
    params = D.channel_params(w.freq_hz)
    ap = torch.from_numpy(w.ap_xyz).cuda()
    foc = torch.from_numpy(w.focal_xyz[None]).cuda()          # [1][1][3]
    gpts = D.grid_points(w.grid)

    def run():
        Hf = D.channel(params, ap, D.list_points(foc, 1), prec="f64")
        r = D.beamform(Hf, "mr", None, w.sigma2, w.p_total, "f64")
        return D.powermap(params, ap[0].contiguous(), r.W[0], gpts, w.sigma2, "f64")
    m = run()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(20):
        m = run()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 20
    aps = w.ap_xyz[0]
    Hf = O.los_channel(w.focal_xyz, aps, w.freq_hz)
    Wm = O.mr_precoder(Hf, w.p_total)
    Hg = O.los_channel(O.grid_points(*[getattr(w.grid, k) for k in ("x0", "y0", "dx", "dy", "z",
                                                                  "nx", "ny")]), aps, w.freq_hz)
    y = m.power.cpu().numpy()
    s = m.sinr.cpu().numpy()
    # the map at the focal point itself: normalised MR gives y = P sum_m |h_m|^2
    Hd = D.channel(params, ap, D.list_points(foc, 1), prec="f64")
    Wd = D.beamform(Hd, "mr", None, w.sigma2, w.p_total, "f64").W[0]
    yf = D.powermap(params, ap[0].contiguous(), Wd, D.list_points(foc[0], 1), w.sigma2,
                    "f64").power.cpu().numpy()[0]
    return {"workload": "focus: M=16 APs on the ceiling (z=3 m) of a 10x10x3 m room, 920 MHz, "
                        "MR at 1 W focused on one point at z=1 m, 64x64 map at z=1 m, FP64",
            "ms_per_call_chain": round(ms, 4),
            "terms": int(w.grid.n * w.M + 2 * w.M),
            "err_db": {"power": db_report(y, O.power_map(Hg, Wm), 1e-9),
                       "snr": db_report(s, O.sinr_map(Hg, Wm, w.sigma2)[0], 1e-9),
                       "focal_point_vs_closed_form_db": float(abs(10 * np.log10(
                           yf / (w.p_total * np.sum(np.abs(Hf) ** 2)))))}}


def paper_phase(D, WL, torch):
    """The paper's ZF on its own workload (5000 Rayleigh channels, K = 8,
    M = 64, gamma 10 dB, sigma 1; Sec. VI-B): every SINR_k must equal the
    target and R_sum = 8 log2 11 = 27.68 bit/symbol.  GPU against the oracle
    and against that closed form, and the MR sum rate against the oracle."""
    import numpy as np
    from oracle import dmimo_oracle as O
    w = WL.paper_workload(seed=0, B=5000)
    H = torch.from_numpy(w.H.astype(np.complex64)).cuda()
    zf = D.beamform(H, "zf", w.gamma_lin, w.sigma2, 0.0, "f32")
    mr = D.beamform(H, "mr", None, w.sigma2, 0.0, "f32")
    torch.cuda.synchronize()
    Hc = w.H.astype(np.complex64).astype(np.complex128)
    idx = np.arange(0, 5000, 50)
    Wz, _ = O.zf_precoder(Hc[idx], w.gamma_lin, w.sigma2, 0.0)
    sz = O.user_sinr(Hc[idx], Wz, w.sigma2)
    Wm = O.mr_precoder(Hc[idx], 0.0)
    sm = O.user_sinr(Hc[idx], Wm, w.sigma2)
    g_sinr = zf.sinr.cpu().numpy()
    rs = zf.rsum.cpu().numpy()
    target = 8 * np.log2(11.0)
    return {"workload": "paper: 5000 Rayleigh channels CN(0,1), K=8, M=64, gamma 10 dB, sigma 1; "
                        "ZF with the constraint of eq. (optim1), MR = H^*",
            "zf_rsum_mean": float(rs.mean()), "zf_rsum_paper": round(target, 4),
            "zf_rsum_max_abs_err": float(np.abs(rs - target).max()),
            "err_db": {"zf_user_sinr_vs_oracle": plain_db(g_sinr[idx], sz),
                       "zf_user_sinr_vs_target": plain_db(g_sinr, np.full(g_sinr.shape, 10.0)),
                       "mr_user_sinr_vs_oracle": plain_db(mr.sinr.cpu().numpy()[idx], sm),
                       "compared": "100 sampled channels vs the oracle; all 5000 vs the 10 dB target"}}


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


def channel_phase(D, WL, torch):
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
    w = WL.room_workload()
    params = D.channel_params(w.freq_hz)
    ap = torch.from_numpy(w.ap_xyz).cuda()
    gpts = D.grid_points(w.grid)
    N, M = w.grid.n, w.M
    out = {"room_f32": run(params, ap, gpts, N, M, "f32", 50),
           "room_f64": run(params, ap, gpts, N, M, "f64", 50)}
    hw = WL.hall_workload()
    hap = torch.from_numpy(hw.ap_xyz).cuda()
    out["hall_f32"] = run(D.channel_params(hw.freq_hz), hap, D.grid_points(hw.grid), hw.grid.n,
                          hw.M, "f32", 5)
    out["workload"] = ("room: 512 x 512 grid x 64 APs (16.8 M terms); hall: 2048 x 2048 grid x "
                       "1024 APs (4.29 G terms); LoS, output H [N][M] in HBM")
    return out


# every file the fused batched kernel is compiled from
BATCHED_SOURCES = ["paper_2304_12745_amd/csrc/batched.hip",
                   "paper_2304_12745_amd/csrc/split16.h",
                   "paper_2304_12745_amd/csrc/kernels.h",
                   "paper_2304_12745_amd/csrc/dmimo_internal.h"]
BATCHED_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "batched_rician_traffic.json")


def batched_bytes(B, K, M, want_W=True):
    """Algorithmic HBM bytes of one fused batched launch: the NLoS draws, the
    antenna and user positions read once, W, p_m, SINR_k, R_sum, l21 and
    info written once."""
    per = K * M * 8 + M * 24 + K * 24 + (K * M * 8 if want_W else 0) + M * 8 + K * 8 + 8 + 8 + 4
    return B * per


def batched_phase(D, WL, torch, event_launches=30):
    """The batched configuration: B independent rooms of K = 16 users and
    M = 256 antennas at 5.8 GHz, Rician channels (K-factor 6 dB, CN(0,1) NLoS
    draws from the seed), ZF at 1 W, -90 dBm, per-user SINR_k and R_sum.

    * ``rician``: the 1024 rooms of the configuration through the fused
      dmimo_beamform_batched (synthesis -> Gram on the matrix cores -> FP64
      solve -> W, p_m, SINR_k) in FP16x3, BF16x3 and FP32; SINR_k of sampled
      deployments against the FP64 oracle chain in dB, and against the
      two-call path (dmimo_channel + dmimo_beamform), which is also timed
      (dmimo_beamform runs the same kernel on the written H: equal bits).
    * ``sweep``: the fused call for B = 2^10 .. 2^17 (the 1024 rooms tiled),
      HBM fraction of the algorithmic bytes (batched_bytes).
    * ``from_h``: dmimo_beamform (ZF at 1 W) of B = 2^17 CN(0,1) channels
      drawn on the device, FP32 and FP16x3, HBM fraction of H read + W and
      the epilogues written; ``gram``: dmimo_gram of the same channels in
      FP32, FP16x3 and BF16x3.
    * ``roofline``: B = 2^17 FP16x3 with W written, from HIP events around
      ``event_launches`` back-to-back launches; traffic from the committed
      counter summary when it matches the sources.
    * ``cpu_oracle``: the oracle chain on the sampled deployments, one core."""
    import numpy as np
    from oracle import dmimo_oracle as O
    K, M = 16, 256

    def timed(fn, reps):
        for _ in range(2):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    w = WL.batched_workload()
    B = w.B
    params = D.channel_params(w.freq_hz, D.CH_RICIAN, w.kappa_lin)
    ap = torch.from_numpy(w.ap_xyz).cuda()
    users = torch.from_numpy(w.user_xyz).cuda()
    nlos = torch.from_numpy(w.nlos).cuda()
    idx = np.arange(0, B, 32)
    t0 = time.perf_counter()
    Ho = np.stack([O.rician_channel(w.user_xyz[b], w.ap_xyz[b], w.freq_hz, w.kappa_lin,
                                    w.nlos[b].astype(np.complex128)) for b in idx])
    Wo, _ = O.zf_precoder(Ho, None, w.sigma2, w.p_total)
    so = O.user_sinr(Ho, Wo, w.sigma2)
    t_oracle = time.perf_counter() - t0
    ric = {}
    for prec in ("f16x3", "bf16x3", "f32"):
        r = D.beamform_batched(params, ap, users, nlos, "zf", None, w.sigma2, w.p_total, prec)
        ms = timed(lambda: D.beamform_batched(params, ap, users, nlos, "zf", None, w.sigma2,
                                              w.p_total, prec, out=r), 20)
        ric[prec] = {"ms": round(ms, 4),
                     "deployments_per_s": round(B / (ms * 1e-3), 1),
                     "G_h_per_s": round(B * K * M / (ms * 1e-3) / 1e9, 2),
                     "hbm_frac": round(batched_bytes(B, K, M) / (ms * 1e-3) / HBM_PEAK, 4),
                     "failed_deployments": int((r.info != 0).sum().item()),
                     "err_db_user_sinr": plain_db(r.sinr.cpu().numpy()[idx], so)}
        if prec in ("f16x3", "f32"):
            # the two-call path: channel to HBM, then ZF from HBM
            pts = D.list_points(users, K)
            H = D.channel(params, ap, pts, nlos=nlos, prec="f32")
            r2 = D.beamform(H, "zf", None, w.sigma2, w.p_total, prec)
            ms_ch = timed(lambda: D.channel(params, ap, pts, nlos=nlos, prec="f32", out=H), 20)
            ms_bf = timed(lambda: D.beamform(H, "zf", None, w.sigma2, w.p_total, prec, out=r2), 20)
            ric[prec]["two_call"] = {"channel_ms": round(ms_ch, 4), "beamform_ms": round(ms_bf, 4),
                                     "ms": round(ms_ch + ms_bf, 4),
                                     "equal_bits": all(torch.equal(getattr(r, n), getattr(r2, n))
                                                       for n in ("W", "p_ant", "l21", "sinr",
                                                                 "rsum", "info"))}
            ric[prec]["err_db_vs_two_call"] = plain_db(r.sinr.cpu().numpy(), r2.sinr.cpu().numpy())
            del H, r2
        del r
    ric["workload"] = ("1024 rooms 20x20x4 m, 16x16 jittered ceiling APs, 16 users at 1.2 m, "
                       "5.8 GHz, Rician K-factor 6 dB with CN(0,1) NLoS draws, ZF at 1 W, "
                       "-90 dBm; one dmimo_beamform_batched launch")
    ric["compared"] = f"per-user SINR_k of {len(idx)} sampled deployments vs the oracle chain"
    torch.cuda.empty_cache()

    sweep = []
    roof = None
    bmax = 1 << 17
    f = bmax // B
    apT = ap.repeat(f, 1, 1).contiguous()
    usT = users.repeat(f, 1, 1).contiguous()
    nlT = nlos.repeat(f, 1, 1).contiguous()
    for prec in ("f16x3", "f32"):
        for e in (10, 12, 14, 16, 17):
            Bs = 1 << e
            a_, u_, n_ = apT[:Bs], usT[:Bs], nlT[:Bs]
            r = D.beamform_batched(params, a_, u_, n_, "zf", None, w.sigma2, w.p_total, prec)
            ms = timed(lambda: D.beamform_batched(params, a_, u_, n_, "zf", None, w.sigma2,
                                                  w.p_total, prec, out=r),
                       20 if Bs <= 1 << 14 else 10)
            sweep.append({"B": Bs, "prec": prec, "ms": round(ms, 4),
                          "deployments_per_s": round(Bs / ms * 1e3, 1),
                          "G_h_per_s": round(Bs * K * M / ms / 1e6, 2),
                          "hbm_frac": round(batched_bytes(Bs, K, M) / (ms * 1e-3) / HBM_PEAK, 4)})
            if e == 17 and prec == "f16x3":
                launch_ms = timed(lambda: D.beamform_batched(params, a_, u_, n_, "zf", None, w.sigma2,
                                                             w.p_total, prec, out=r), event_launches)
                byts = batched_bytes(Bs, K, M)
                khash = _src_hash(BATCHED_SOURCES)
                roof = {"bound": "hbm",
                        "kernel": "beamform_batched_kernel<1, false> (FP16x3), 131072 Rician rooms, W written",
                        "achieved": round(byts / (launch_ms * 1e-3) / 1e9, 1),
                        "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                        "frac": round(byts / (launch_ms * 1e-3) / HBM_PEAK, 4),
                        "traffic": load_traffic(khash, BATCHED_TRAFFIC_FILE),
                        "launch_ms": round(launch_ms, 5), "launches_timed": event_launches,
                        "algorithmic_bytes_per_launch": byts, "source_hash": khash}
            del r
    del apT, usT, nlT
    torch.cuda.empty_cache()
    # dmimo_beamform from H (8 < K <= 16, M <= 256: the same kernel, channel loaded)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(3)
    Hr = torch.complex(torch.randn(bmax, K, M, generator=gen, device="cuda"),
                       torch.randn(bmax, K, M, generator=gen, device="cuda")) * (0.5 ** 0.5)
    from_h = {"workload": f"dmimo_beamform ZF at 1 W of {bmax} CN(0,1) channels K={K} M={M}, "
                          "sigma2 = 1, H resident; hbm_frac of H read + W, p_m, SINR_k and "
                          "the scalars written"}
    hbytes = bmax * (K * M * 16 + M * 8 + K * 8 + 20)
    for prec in ("f32", "f16x3"):
        r = D.beamform(Hr, "zf", None, 1.0, 1.0, prec)
        ms = timed(lambda: D.beamform(Hr, "zf", None, 1.0, 1.0, prec, out=r), 10)
        from_h[prec] = {"ms": round(ms, 4), "hbm_frac": round(hbytes / (ms * 1e-3) / HBM_PEAK, 4),
                        "failed_deployments": int((r.info != 0).sum().item())}
        del r
    # dmimo_gram of the same channels (H read, G written)
    gram = {"workload": f"dmimo_gram of the same {bmax} channels; hbm_frac of H read + G written"}
    gbytes = bmax * (K * M * 8 + K * K * 8)
    for prec in ("f32", "f16x3", "bf16x3"):
        G = D.gram(Hr, prec)
        ms = timed(lambda: D.gram(Hr, prec, out=G), 10)
        gram[prec] = {"ms": round(ms, 4), "hbm_frac": round(gbytes / (ms * 1e-3) / HBM_PEAK, 4)}
        del G
    del Hr
    torch.cuda.empty_cache()
    return {"rician": ric,
            "from_h": from_h,
            "gram": gram,
            "sweep_workload": "fused dmimo_beamform_batched, B rooms (the 1024 tiled) x K=16 x M=256, "
                              "Rician, ZF at 1 W, W written; hbm_frac of the algorithmic bytes "
                              "(NLoS + positions read, W + p_m + SINR + R_sum written)",
            "sweep": sweep,
            "roofline": roof,
            "cpu_oracle": {"value": round(len(idx) / t_oracle, 2), "unit": "deployments/s",
                           "cores": 1, "kind": "oracle",
                           "sample": f"{len(idx)} deployments: rician_channel + zf_precoder + user_sinr"}}


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


def pa_phase(w, D, WL, torch):
    """The PA-consumption-aware precoder (eq. optim1 by normalised PGD, lambda =
    1/15, 5000 iterations) on the benchmark room: the step's K = 8 users, SINR
    targets 10 dB, noise -90 dBm.  Reports its PCG against ZF with the same
    targets, the APs it switches off and the SINR range; times the precoder
    and the 512 x 512 power + SINR map of the sparse W; then the precoder's
    throughput over 1024 user draws in the same room (one launch)."""
    import numpy as np

    K, M, N = w.K, w.M, w.grid.n
    params = D.channel_params(w.freq_hz)
    gpts = D.grid_points(w.grid)
    ap0 = torch.from_numpy(w.ap_xyz[0]).cuda().contiguous()
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



if __name__ == "__main__":
    main()
