"""GPU parity: every entry point of libdmimo vs the FP64 oracle.

Both sides take the same seeded inputs.  Complex64 inputs are rounded once
and the oracle receives the rounded values, upcast.  Tolerances:

* power / SINR maps: 0.01 dB for FP32, 0.1 dB for the mixed FP16/BF16 x3
  paths, with the -60 dB floor rule (oracle/dberror.py).  FP64 maps use 1e-9 dB.
* per-user SINR: plain dB error, same budgets.
* channel terms, Gram and W: relative bounds derived from the arithmetic:
  - FP32 channel: |dh|/|h| <= 2e-6.  That is the FP32 amplitude seed (2^-22)
    plus the hardware sin/cos in revolutions (a few 2^-22) plus two roundings.
  - FP32 Gram: |dG_kj| <= 1e-5 sqrt(G_kk G_jj).  That is an FP32 sum of M
    products (M <= 1024) with a margin.
  - ZF W: 1e-4 relative in Frobenius norm (FP32 Gram error times cond(G) <= 100).
  - FP64 paths: 1e-11 relative.
"""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import dmimo_oracle as O  # noqa: E402
from oracle import dberror  # noqa: E402
from paper_2304_12745_amd import workloads as WL  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def D():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_2304_12745_amd import dmimo
    dmimo.lib()
    return dmimo


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(x, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def c64(x):
    return np.asarray(x).astype(np.complex64)


def rel_err(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


def grid_pts(g):
    return O.grid_points(g.x0, g.y0, g.dx, g.dy, g.z, g.nx, g.ny)


MAP_TOL = {"f32": 0.01, "f16x3": 0.1, "bf16x3": 0.1}


def check_db(y, ref, tol, floor_rel=1e-6, what=""):
    s = dberror.summary(y, ref, tol, floor_rel)
    say(f"    {what}: max {s['max_db']:.2e} dB  p99 {s['p99_db']:.2e} dB  "
        f"below floor {s['n_below_floor']}/{s['n']}  fail {s['n_fail']}")
    assert s["n_fail"] == 0, s
    return s


# ---------------------------------------------------------------------------
# dmimo_channel
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("M", [64, 37, 1, 5])
def test_channel_los_grid(D, prec, M):
    say(f"channel LoS grid prec={prec} M={M}")
    rng = np.random.default_rng(100 + M)
    aps = WL.uniform_positions(rng, M, 20, 20, 4.0)
    g = WL.Grid(0.0, 0.0, 20 / 23, 20 / 9, 1.2, 23, 9)      # N = 207: ragged
    f = 3.5e9
    H = D.channel(D.channel_params(f), dev(aps[None]), D.grid_points(g), prec=prec)
    h = host(H)[0]
    ref = O.los_channel(grid_pts(g), aps, f)
    tol = 2e-6 if prec == "f32" else 1e-11
    e = np.max(np.abs(h - ref) / np.abs(ref))
    say(f"    max |dh|/|h| = {e:.3e}")
    assert e <= tol


# more rows than one grid-stride step covers (65536 rows for M >= 33, 524288
# for M = 5), the step crossing deployments: sampled rows against the oracle
@pytest.mark.parametrize("M,B,nx,ny,kind,prec", [(64, 3, 250, 160, "grid", "f32"),
                                                 (64, 3, 250, 160, "grid", "f64"),
                                                 (5, 2, 600, 500, "grid", "f32"),
                                                 (64, 3, 40000, 1, "list", "f32"),
                                                 (37, 2, 50000, 1, "list", "f32")])
def test_channel_grid_stride_wrap(D, M, B, nx, ny, kind, prec):
    say(f"channel {kind} B={B} N={nx * ny} M={M} prec={prec}")
    rng = np.random.default_rng(M + 10 * B + nx)
    aps = np.stack([WL.uniform_positions(rng, M, 20, 20, 4.0) for _ in range(B)])
    f = 3.5e9
    if kind == "grid":
        g = WL.Grid(0.0, 0.0, 20 / nx, 20 / ny, 1.2, nx, ny)
        pts = np.broadcast_to(grid_pts(g), (B, nx * ny, 3))
        desc = D.grid_points(g)
    else:
        pts = np.stack([WL.uniform_positions(rng, nx, 20, 20, 1.2) for _ in range(B)])
        desc = D.list_points(dev(pts), nx)
    H = host(D.channel(D.channel_params(f), dev(aps), desc, prec=prec))
    assert H.shape == (B, nx * ny, M)
    tol = 2e-6 if prec == "f32" else 1e-11
    for b in range(B):
        rows = np.concatenate([[0, nx * ny - 1], rng.choice(nx * ny, 200, replace=False)])
        ref = O.los_channel(pts[b][rows], aps[b], f)
        e = np.max(np.abs(H[b][rows] - ref) / np.abs(ref))
        assert e <= tol, (b, e)


# rows wider than 64 antennas: one deployment holds its antenna coordinates
# in LDS (M <= 2048), several deployments or more antennas read them from HBM
@pytest.mark.parametrize("M,B,kind", [(100, 1, "grid"), (2048, 1, "grid"), (2049, 1, "grid"),
                                      (300, 2, "grid"), (1024, 1, "list")])
def test_channel_wide_rows(D, M, B, kind):
    say(f"channel wide rows {kind} B={B} M={M}")
    rng = np.random.default_rng(M + B)
    aps = np.stack([WL.uniform_positions(rng, M, 50, 50, 5.0) for _ in range(B)])
    f = 5.8e9
    if kind == "grid":
        g = WL.Grid(0.0, 0.0, 50 / 41, 50 / 37, 1.0, 41, 37)
        pts = np.broadcast_to(grid_pts(g), (B, g.nx * g.ny, 3))
        desc = D.grid_points(g)
    else:
        pts = np.stack([WL.uniform_positions(rng, 1500, 50, 50, 1.0) for _ in range(B)])
        desc = D.list_points(dev(pts), 1500)
    for prec, tol in (("f32", 2e-6), ("f64", 1e-11)):
        H = host(D.channel(D.channel_params(f), dev(aps), desc, prec=prec))
        for b in range(B):
            ref = O.los_channel(pts[b], aps[b], f)
            e = np.max(np.abs(H[b] - ref) / np.abs(ref))
            assert e <= tol, (prec, b, e)


# one deployment with wide rows and at least 4096 points takes the row-per-
# workgroup kernel (16 consecutive rows per workgroup, 16-byte stores of
# antenna pairs): a grid of 4801 points (the last workgroup holds one row) and
# a list of 4100, every term against the oracle
@pytest.mark.parametrize("kind,n", [("grid", 4801), ("list", 4100)])
def test_channel_rows_per_workgroup(D, kind, n):
    say(f"channel rows per workgroup: {kind} N={n} M=1024")
    rng = np.random.default_rng(n)
    M, f = 1024, 5.8e9
    aps = WL.uniform_positions(rng, M, 50, 50, 5.0)
    if kind == "grid":
        g = WL.Grid(0.0, 0.0, 50 / 4801, 50.0, 1.0, 4801, 1)
        pts, desc = grid_pts(g), D.grid_points(g)
    else:
        pts = WL.uniform_positions(rng, n, 50, 50, 1.0)
        desc = D.list_points(dev(pts[None]), n)
    H = host(D.channel(D.channel_params(f), dev(aps[None]), desc, prec="f32"))[0]
    ref = O.los_channel(pts, aps, f)
    e = np.max(np.abs(H - ref) / np.abs(ref))
    say(f"    max |dh|/|h| = {e:.2e}")
    assert e <= 2e-6


# the materialised channels bench.py times, in the same launch configuration:
# the room's 512 x 512 grid x 64 APs (four antennas per lane) and the hall's
# 2048 x 2048 grid x 1024 APs (34.4 GB; antenna coordinates in LDS); sampled
# rows against the oracle
@pytest.mark.parametrize("name", ["room", "hall"])
def test_channel_bench_configuration_sampled(D, name):
    import torch
    say(f"channel materialised, bench configuration: {name}")
    w = WL.room_workload() if name == "room" else WL.hall_workload()
    g, M = w.grid, w.M
    H = D.channel(D.channel_params(w.freq_hz), dev(w.ap_xyz), D.grid_points(g), prec="f32")
    assert tuple(H.shape) == (1, g.n, M)
    rng = np.random.default_rng(77)
    rows = np.concatenate([[0, g.n - 1, g.nx - 1, g.nx], rng.choice(g.n, 300, replace=False)])
    Hs = H[0][torch.from_numpy(rows).to(H.device)].cpu().numpy()
    del H
    torch.cuda.empty_cache()
    ref = O.los_channel(grid_pts(g)[rows], w.ap_xyz[0], w.freq_hz)
    e = np.max(np.abs(Hs - ref) / np.abs(ref))
    say(f"    max |dh|/|h| over {rows.size} rows: {e:.2e}")
    assert e <= 2e-6


def test_channel_los_list_batched(D):
    say("channel LoS list, B=3")
    rng = np.random.default_rng(7)
    B, K, M = 3, 5, 40
    aps = np.stack([WL.uniform_positions(rng, M, 10, 10, 3.0) for _ in range(B)])
    users = np.stack([WL.uniform_positions(rng, K, 10, 10, 1.0) for _ in range(B)])
    f = 0.92e9
    U = dev(users)
    H = host(D.channel(D.channel_params(f), dev(aps), D.list_points(U, K), prec="f32"))
    for b in range(B):
        ref = O.los_channel(users[b], aps[b], f)
        assert np.max(np.abs(H[b] - ref) / np.abs(ref)) <= 2e-6


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_channel_rician(D, prec):
    say(f"channel Rician prec={prec}")
    w = WL.batched_workload(B=6, K=16, side=16)
    f = w.freq_hz
    U = dev(w.user_xyz)
    H = host(D.channel(D.channel_params(f, D.CH_RICIAN, w.kappa_lin), dev(w.ap_xyz),
                       D.list_points(U, 16), nlos=dev(w.nlos), prec=prec))
    tol = 2e-6 if prec == "f32" else 1e-11
    for b in range(6):
        ref = O.rician_channel(w.user_xyz[b], w.ap_xyz[b], f, w.kappa_lin,
                               w.nlos[b].astype(np.complex128))
        # relative to the path amplitude (the Rician sum itself can be near zero)
        amp = np.abs(O.los_channel(w.user_xyz[b], w.ap_xyz[b], f))
        e = np.max(np.abs(H[b] - ref) / amp)
        assert e <= 3 * tol, e


def test_channel_near_field_clamp(D):
    say("channel near-field clamp")
    f = 1e9
    aps = np.array([[[0.0, 0.0, 0.0], [1.0, 2.0, 3.0]]])
    pts = np.array([[[0.0, 0.0, 0.0]]])
    H = host(D.channel(D.channel_params(f), dev(aps), D.list_points(dev(pts), 1), prec="f64"))
    ref = O.los_channel(pts[0], aps[0], f)
    np.testing.assert_allclose(H[0], ref, rtol=1e-12)
    assert abs(H[0, 0, 0]) == pytest.approx(1.0, rel=1e-12)


# the FP64 phase at every fraction of a turn: one antenna, points on a line at
# distances lambda (1 + i/4096) and next to each eighth of a turn.  With fewer
# than two revolutions the oracle's own phase rounding stays near 3e-15, so the
# sine and cosine of the fractional revolution are held to 2e-14 here (the
# other FP64 channel tests allow 1e-11 for distances of thousands of turns).
def test_channel_f64_phase_every_fraction(D):
    say("channel FP64 phase over one turn")
    f = 3.5e9
    lam = O.wavelength(f)
    frac = np.arange(4096) / 4096.0
    edges = np.arange(1, 17) / 8.0
    frac = np.concatenate([frac, np.nextafter(edges, 0.0) - 1.0, np.nextafter(edges, 3.0) - 1.0])
    d = lam * (1.0 + frac)
    pts = np.stack([d, np.zeros_like(d), np.zeros_like(d)], axis=1)[None]
    aps = np.zeros((1, 1, 3))
    H = host(D.channel(D.channel_params(f), dev(aps), D.list_points(dev(pts), d.size), prec="f64"))
    ref = O.los_channel(pts[0], aps[0], f)
    e = np.max(np.abs(H[0] - ref) / np.abs(ref))
    say(f"    max |dh|/|h| over {d.size} fractions: {e:.2e}")
    assert e <= 2e-14


# ---------------------------------------------------------------------------
# dmimo_gram
# ---------------------------------------------------------------------------

# |dG_kj| / sqrt(G_kk G_jj): FP32 sums; FP16 x3 splits every value to
# ~2^-22 and drops lo*lo (~2^-22); BF16 x3 splits to ~2^-17.
GRAM_TOL = {"f64": 1e-12, "f32": 1e-5, "f16x3": 1e-5, "bf16x3": 1e-4}


@pytest.mark.parametrize("prec", ["f32", "f64", "f16x3", "bf16x3"])
@pytest.mark.parametrize("K,M", [(8, 64), (16, 256), (5, 37), (32, 1024), (17, 100), (1, 3)])
def test_gram(D, prec, K, M):
    say(f"gram prec={prec} K={K} M={M}")
    rng = np.random.default_rng(K * 1000 + M)
    B = 7
    H = WL.complex_normal(rng, (B, K, M)) * 10.0 ** rng.uniform(-4, 1)
    if prec != "f64":
        H = c64(H)
    G = host(D.gram(dev(H), prec=prec))
    ref = O.gram(H.astype(np.complex128))
    d = np.sqrt(np.abs(np.einsum("bkk->bk", ref)))
    scale = d[:, :, None] * d[:, None, :]
    e = np.max(np.abs(G - ref) / scale)
    say(f"    max |dG|/sqrt(GkkGjj) = {e:.3e}")
    assert e <= GRAM_TOL[prec]
    # exactly Hermitian, real diagonal
    np.testing.assert_array_equal(G, np.conj(np.swapaxes(G, 1, 2)))


# The persistent Gram kernel (four workgroups per CU) takes MIX at K M > 512
# and FP32 at 12 < K <= 16, 128 < M <= 256 (the last four shapes stay on the
# VALU kernel in FP32, two of them just past its boundary): more deployments
# than workgroups, antenna counts on
# and past the boundaries of the waves' 64-antenna shares, deployments whose
# scales differ by 10^5 (the FP16 scale is per deployment) and an all-zero one
@pytest.mark.parametrize("prec", ["f32", "f16x3", "bf16x3"])
@pytest.mark.parametrize("B,K,M", [(1500, 16, 256), (1100, 13, 129), (3, 16, 192), (5, 14, 200),
                                   (4, 4, 256), (3, 9, 65), (6, 12, 200), (6, 16, 128)])
def test_gram_batched_kernel(D, prec, B, K, M):
    say(f"gram (persistent kernel) prec={prec} B={B} K={K} M={M}")
    rng = np.random.default_rng(B + 10 * K + 100 * M)
    H = WL.complex_normal(rng, (B, K, M)) * 10.0 ** rng.uniform(-4, 1, (B, 1, 1))
    H[1] = 0.0
    H = c64(H)
    G = host(D.gram(dev(H), prec=prec))
    assert not np.any(G[1])
    ok = np.arange(B) != 1
    ref = O.gram(H[ok].astype(np.complex128))
    d = np.sqrt(np.abs(np.einsum("bkk->bk", ref)))
    e = np.max(np.abs(G[ok] - ref) / (d[:, :, None] * d[:, None, :]))
    say(f"    max |dG|/sqrt(GkkGjj) = {e:.3e}")
    assert e <= GRAM_TOL[prec]
    np.testing.assert_array_equal(G, np.conj(np.swapaxes(G, 1, 2)))


# ---------------------------------------------------------------------------
# dmimo_beamform
# ---------------------------------------------------------------------------

def _check_beamform(D, H, precoder, gamma, sigma2, p_total, prec, sinr_tol_db, w_tol):
    Hd = dev(H)
    r = D.beamform(Hd, precoder, gamma, sigma2, p_total, prec)
    W = host(r.W)
    Hc = H.astype(np.complex128)
    if precoder == "zf":
        Wr, sing = O.zf_precoder(Hc, gamma, sigma2, p_total)
        assert not sing.any()
    elif precoder == "mr":
        Wr = O.mr_precoder(Hc, p_total)
    else:
        Wr = O.mr_phase_precoder(Hc, p_total)
    np.testing.assert_array_equal(host(r.info), 0)
    ew = np.max(np.linalg.norm(W - Wr, axis=(1, 2)) / np.linalg.norm(Wr, axis=(1, 2)))
    say(f"    W rel err {ew:.2e}")
    assert ew <= w_tol
    np.testing.assert_allclose(host(r.p_ant), O.antenna_power(Wr), rtol=10 * w_tol,
                               atol=10 * w_tol * np.max(O.antenna_power(Wr)))
    np.testing.assert_allclose(host(r.l21), O.l21_norm(Wr), rtol=10 * w_tol)
    sinr_ref = O.user_sinr(Hc, Wr, sigma2)
    sinr = host(r.sinr)
    e = np.max(np.abs(10 * np.log10(sinr / sinr_ref)))
    say(f"    SINR max dB err {e:.2e}")
    assert e <= sinr_tol_db
    rs = host(r.rsum)
    np.testing.assert_allclose(rs, O.sum_rate(sinr_ref), rtol=1e-3)
    return r


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_beamform_paper_zf_sum_rate(D, prec):
    say(f"beamform ZF, paper setting, prec={prec}")
    w = WL.paper_workload(seed=0, B=256)
    H = w.H if prec == "f64" else c64(w.H)
    r = _check_beamform(D, H, "zf", w.gamma_lin, 1.0, 0.0, prec,
                        0.01 if prec == "f32" else 1e-8, 1e-4 if prec == "f32" else 1e-10)
    rs = host(r.rsum)
    # Sec. VI-B: the target sum rate at K=8, gamma=10 dB is 27.68 bits/symbol
    assert np.all(np.abs(rs - 27.68) < 0.005)


@pytest.mark.parametrize("precoder", ["mr", "mr_phase"])
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_beamform_mr_paper(D, precoder, prec):
    say(f"beamform {precoder} prec={prec}")
    w = WL.paper_workload(seed=1, B=64)
    H = w.H if prec == "f64" else c64(w.H)
    _check_beamform(D, H, precoder, None, 1.0, 0.0, prec, 0.01 if prec == "f32" else 1e-8,
                    1e-6 if prec == "f32" else 1e-12)
    _check_beamform(D, H, precoder, None, 1.0, 2.0, prec, 0.01 if prec == "f32" else 1e-8,
                    1e-6 if prec == "f32" else 1e-12)


def _room_users(w):
    return O.los_channel(w.user_xyz[0], w.ap_xyz[0], w.freq_hz)[None]


def test_beamform_room_zf_total_power(D):
    say("beamform ZF room (K=8, M=64, 1 W, -90 dBm)")
    w = WL.room_workload(nx=8, ny=8)
    H = c64(_room_users(w))
    r = _check_beamform(D, H, "zf", None, w.sigma2, 1.0, "f32", 0.01, 1e-4)
    assert host(r.p_ant).sum() == pytest.approx(1.0, rel=1e-5)


@pytest.mark.parametrize("prec", ["f32", "f16x3", "bf16x3"])
def test_beamform_batched_rician_zf(D, prec):
    # K = 16, M = 256: dmimo_beamform runs the persistent batched kernel with H
    # given (Gram on the matrix cores in the precision asked for, FP64
    # inverse); SINR within 0.01 dB (FP32) / 0.1 dB (mixed)
    say(f"beamform ZF batched Rician (K=16, M=256), Gram {prec}")
    w = WL.batched_workload(B=16)
    Hc = np.stack([O.rician_channel(w.user_xyz[b], w.ap_xyz[b], w.freq_hz, w.kappa_lin,
                                    w.nlos[b].astype(np.complex128)) for b in range(16)])
    _check_beamform(D, c64(Hc), "zf", None, w.sigma2, 1.0, prec, MAP_TOL[prec],
                    1e-4 if prec != "bf16x3" else 1e-2)


# dmimo_beamform at the batched sweep's shape: B deployments of K = 16,
# M = 256 with H drawn on the device (the seeded draw of the bench's from-H
# leg), ZF at 1 W, on the persistent batched kernel; sampled deployments
# against the oracle.  The noise is sigma2 = 1 here (the launch is the same): at the
# sweep's -90 dBm with unit channels the SINR would measure the FP32 rounding
# interference of W, not the precoder.
@pytest.mark.parametrize("B,prec", [(1024, "f32"), (131072, "f32"), (131072, "f16x3")])
def test_beamform_batched_sweep_configuration_sampled(D, B, prec):
    import torch
    say(f"beamform ZF, batched sweep configuration B={B} prec={prec}")
    K, M = 16, 256
    gen = torch.Generator(device="cuda")
    gen.manual_seed(3)
    bmax = 1 << 17
    H = torch.complex(torch.randn(bmax, K, M, generator=gen, device="cuda"),
                      torch.randn(bmax, K, M, generator=gen, device="cuda")) * (0.5 ** 0.5)
    Hb = H[:B]
    r = D.beamform(Hb, "zf", None, 1.0, 1.0, prec)
    rng = np.random.default_rng(B)
    pick = np.concatenate([[0, B - 1], rng.choice(B, 14, replace=False)])
    idx = torch.from_numpy(pick).to(H.device)
    Hs = Hb[idx].cpu().numpy().astype(np.complex128)
    W = r.W[idx].cpu().numpy()
    sinr = r.sinr[idx].cpu().numpy()
    assert not np.any(r.info[idx].cpu().numpy())
    del H, Hb, r
    torch.cuda.empty_cache()
    Wr, sing = O.zf_precoder(Hs, None, 1.0, 1.0)
    assert not sing.any()
    ew = np.max(np.linalg.norm(W - Wr, axis=(1, 2)) / np.linalg.norm(Wr, axis=(1, 2)))
    es = np.max(np.abs(10 * np.log10(sinr / O.user_sinr(Hs, Wr, 1.0))))
    say(f"    W rel err {ew:.2e}, SINR max dB err {es:.2e}")
    assert ew <= 1e-4 and es <= MAP_TOL[prec]


# dmimo_gram at the bench's full size: the B = 2^17 CN(0,1) channels of its
# from-H leg (K = 16, M = 256, the same seeded device draw), each precision on
# the persistent Gram kernel; sampled deployments against the oracle
@pytest.mark.parametrize("prec", ["f32", "f16x3", "bf16x3"])
def test_gram_bench_configuration_sampled(D, prec):
    import torch
    say(f"gram, B = 131072 CN(0,1) channels K=16 M=256, prec={prec}")
    K, M, B = 16, 256, 1 << 17
    gen = torch.Generator(device="cuda")
    gen.manual_seed(3)
    H = torch.complex(torch.randn(B, K, M, generator=gen, device="cuda"),
                      torch.randn(B, K, M, generator=gen, device="cuda")) * (0.5 ** 0.5)
    G = D.gram(H, prec)
    rng = np.random.default_rng(17)
    pick = np.concatenate([[0, B - 1], rng.choice(B, 14, replace=False)])
    idx = torch.from_numpy(pick).to(H.device)
    Hs = H[idx].cpu().numpy().astype(np.complex128)
    Gs = G[idx].cpu().numpy()
    del H, G
    torch.cuda.empty_cache()
    ref = O.gram(Hs)
    d = np.sqrt(np.abs(np.einsum("bkk->bk", ref)))
    e = np.max(np.abs(Gs - ref) / (d[:, :, None] * d[:, None, :]))
    say(f"    max |dG|/sqrt(GkkGjj) = {e:.3e}")
    assert e <= GRAM_TOL[prec]
    np.testing.assert_array_equal(Gs, np.conj(np.swapaxes(Gs, 1, 2)))


@pytest.mark.parametrize("prec", ["f16x3", "bf16x3"])
def test_beamform_paper_zf_mixed(D, prec):
    # K <= 8 and M <= 256: G is formed in FP64 inside the one-pass kernel in
    # every mode, so the mixed modes give the FP32 result bit for bit
    say(f"beamform ZF, paper setting, prec {prec}")
    w = WL.paper_workload(seed=0, B=256)
    r = _check_beamform(D, c64(w.H), "zf", w.gamma_lin, 1.0, 0.0, prec, MAP_TOL[prec],
                        1e-4 if prec != "bf16x3" else 1e-2)
    assert np.all(np.abs(host(r.rsum) - 27.68) < 0.005)
    r32 = D.beamform(dev(c64(w.H)), "zf", w.gamma_lin, 1.0, 0.0, "f32")
    np.testing.assert_array_equal(host(r.W), host(r32.W))


# one-pass kernel: K <= 8 with M <= 256 (M <= 128 in FP64), ragged tiles and
# the limits; (8, 129) and (8, 257) fall just outside it (FP64 / every mode)
@pytest.mark.parametrize("K,M", [(1, 1), (3, 3), (5, 37), (8, 128), (8, 129), (7, 193), (8, 256),
                                 (8, 257), (32, 64), (17, 300)])
def test_beamform_shapes(D, K, M):
    say(f"beamform ZF/MR shapes K={K} M={M}")
    rng = np.random.default_rng(K + 7 * M)
    H = WL.complex_normal(rng, (3, K, M))
    _check_beamform(D, H, "zf", np.linspace(1, 4, K), 0.5, 0.0, "f64", 1e-7, 1e-9)
    _check_beamform(D, c64(H), "mr", None, 0.5, 1.0, "f32", 0.01, 1e-6)


# ZF of few deployments with many antennas runs on the wide path (B <= 64 and
# at least 8 tiles of 64 antennas: G^-1 once, tiles in parallel workgroups,
# gain shares summed in tile order); B = 65 and M = 448 fall outside it
@pytest.mark.parametrize("B,K,M,prec", [(1, 32, 1024, "f32"), (2, 16, 512, "f32"), (3, 20, 700, "f64"),
                                        (1, 5, 449, "f32"), (64, 8, 512, "f32"), (65, 8, 512, "f32"),
                                        (2, 12, 448, "f32"), (1, 16, 600, "f16x3")])
def test_beamform_wide_zf(D, B, K, M, prec):
    say(f"beamform ZF wide B={B} K={K} M={M} prec={prec}")
    rng = np.random.default_rng(B + K + M)
    H = WL.complex_normal(rng, (B, K, M))
    Hin = H if prec == "f64" else c64(H)
    tol = {"f64": (1e-7, 1e-9), "f32": (0.01, 1e-4), "f16x3": (MAP_TOL["f16x3"], 1e-4)}[prec]
    _check_beamform(D, Hin, "zf", np.linspace(1, 4, K), 0.5, 0.0, prec, tol[0], tol[1])
    _check_beamform(D, Hin, "zf", None, 0.5, 1.0, prec, tol[0], tol[1])


# MR and equal-gain MR of few deployments with many antennas take the same
# wide path (MR: ||H||_F^2 from per-tile shares summed in tile order; no norm
# for p_total <= 0 or equal gain); B = 65 and M = 448 fall outside it
@pytest.mark.parametrize("precoder", ["mr", "mr_phase"])
@pytest.mark.parametrize("B,K,M,prec", [(1, 32, 1024, "f32"), (3, 20, 700, "f64"), (1, 5, 449, "f32"),
                                        (64, 8, 512, "f32"), (65, 8, 512, "f32"), (2, 12, 448, "f32"),
                                        (1, 16, 4096, "f32"), (2, 3, 1000, "f16x3")])
def test_beamform_wide_mr(D, precoder, B, K, M, prec):
    say(f"beamform {precoder} wide B={B} K={K} M={M} prec={prec}")
    rng = np.random.default_rng(B * K + M)
    H = WL.complex_normal(rng, (B, K, M))
    Hin = H if prec == "f64" else c64(H)
    tol = (1e-8, 1e-12) if prec == "f64" else (0.01, 1e-6)
    for p_total in (2.0, 0.0):
        _check_beamform(D, Hin, precoder, None, 0.5, p_total, prec, tol[0], tol[1])


def test_beamform_hall_mr_wide_path(D):
    say("beamform MR, hall deployment (wide path)")
    w = WL.hall_workload()
    H = c64(O.los_channel(w.user_xyz[0], w.ap_xyz[0], w.freq_hz)[None])
    r = _check_beamform(D, H, "mr", None, w.sigma2, 1.0, "f32", 0.01, 1e-6)
    assert abs(float(np.sum(np.abs(host(r.W)) ** 2)) - 1.0) < 1e-5


# several precoders of the same channels in one call equal one call per
# precoder bit for bit: the one-pass kernel with precoder p on grid row p
# (FP32, FP64, FP16x3 Gram mode; ragged M; a singular deployment for ZF), and
# the per-precoder sequence elsewhere (K = 12; the wide path at M = 600)
@pytest.mark.parametrize("B,K,M,prec", [(1, 8, 64, "f32"), (5, 3, 37, "f64"), (7, 8, 256, "f16x3"),
                                        (3, 12, 100, "f32"), (2, 6, 600, "f32")])
def test_beamform_multi_equals_single_calls(D, B, K, M, prec):
    import torch
    say(f"beamform_multi B={B} K={K} M={M} prec={prec}")
    rng = np.random.default_rng(B * 100 + K + M)
    H = WL.complex_normal(rng, (B, K, M))
    if B == 5:
        H[0, 1] = H[0, 0]                      # ZF fails on deployment 0 only
    Hd = dev(H if prec == "f64" else c64(H))
    pcs = ["mr", "zf", "mr_phase", "zf"]
    gamma = np.linspace(1, 3, K)
    for p_total in (1.0, 0.0):
        r = D.beamform_multi(Hd, pcs, gamma, 0.5, p_total, prec)
        assert tuple(r.W.shape) == (len(pcs), B, K, M)
        for i, pc in enumerate(pcs):
            one = D.beamform(Hd, pc, gamma, 0.5, p_total, prec)
            for x, y in ((r.W[i], one.W), (r.p_ant[i], one.p_ant), (r.l21[i], one.l21),
                         (r.sinr[i], one.sinr), (r.rsum[i], one.rsum), (r.info[i], one.info)):
                assert torch.equal(x, y), (pc, p_total)
    if B == 5:
        assert host(r.info)[1, 0] > 0 and np.all(host(r.info)[1, 1:] == 0)
    # W alone (every optional output NULL)
    w_only = D.beamform_multi(Hd, pcs, gamma, 0.5, 1.0, prec, outputs=False)
    for i, pc in enumerate(pcs):
        assert torch.equal(w_only.W[i], D.beamform(Hd, pc, gamma, 0.5, 1.0, prec).W), pc


@pytest.mark.parametrize("B,K,M,prec,d_min", [
    (3, 4, 64, "f32", 0.0),        # one launch, synthesis in the precoder kernel
    (2, 8, 256, "bf16x3", 2.5),    # one launch, near-field clamp on some terms
    (2, 8, 128, "f64", 2.5),       # one launch, FP64 terms
    (2, 12, 300, "f32", 0.0),      # channel kernel, then the precoders
    (1, 9, 600, "f64", 0.0),       # channel kernel, then the wide path
])
def test_beamform_users_equals_channel_then_multi(D, B, K, M, prec, d_min):
    import torch
    say(f"beamform_users B={B} K={K} M={M} prec={prec} d_min={d_min}")
    rng = np.random.default_rng(B * 1000 + K * 10 + M)
    aps = np.stack([WL.uniform_positions(rng, M, 12, 12, 3.0) for _ in range(B)])
    users = np.stack([WL.uniform_positions(rng, K, 12, 12, 1.5) for _ in range(B)])
    params = D.channel_params(3.5e9, D.CH_LOS, 0.0, d_min)
    ap_d, us_d = dev(aps), dev(users)
    pcs = ["mr", "zf", "mr_phase"]
    gamma = np.linspace(1, 2, K)
    ch = "f64" if prec == "f64" else "f32"
    H_ref = D.channel(params, ap_d, D.list_points(us_d, K), prec=ch)
    ref = D.beamform_multi(H_ref, pcs, gamma, 1e-10, 0.0, prec)
    r = D.beamform_users(params, ap_d, us_d, pcs, gamma, 1e-10, 0.0, prec)
    assert torch.equal(r.H, H_ref)
    for x, y in ((r.W, ref.W), (r.p_ant, ref.p_ant), (r.l21, ref.l21), (r.sinr, ref.sinr),
                 (r.rsum, ref.rsum), (r.info, ref.info)):
        assert torch.equal(x, y)
    # the channel itself against the oracle's LoS definition
    Ho = np.stack([O.los_channel(users[b], aps[b], 3.5e9, d_min=d_min) for b in range(B)])
    err = np.abs(host(r.H) - Ho).max() / np.abs(Ho).max()
    assert err < (1e-12 if prec == "f64" else 2e-6)
    # second call into the same outputs, precoders in another order, W alone
    r2 = D.beamform_users(params, ap_d, us_d, ["zf", "mr"], gamma, 1e-10, 1.0, prec,
                          outputs=False)
    ref2 = D.beamform_multi(H_ref, ["zf", "mr"], gamma, 1e-10, 1.0, prec, outputs=False)
    assert torch.equal(r2.H, H_ref) and torch.equal(r2.W, ref2.W)


@pytest.mark.parametrize("prec", ["f32", "f16x3"])
def test_beamform_users_room_step(D, prec):
    # the room's users and APs at the benchmark's precoder settings (MR and ZF
    # at 1 W), against the separate calls and the oracle's channel
    import torch
    say(f"beamform_users room K=8 M=64 prec={prec}")
    w = WL.room_workload(nx=8, ny=8)
    params = D.channel_params(w.freq_hz)
    ap_d, us_d = dev(w.ap_xyz), dev(w.user_xyz)
    H_ref = D.channel(params, ap_d, D.list_points(us_d, w.K), prec="f32")
    ref = D.beamform_multi(H_ref, ["mr", "zf"], None, w.sigma2, w.p_total, prec)
    r = D.beamform_users(params, ap_d, us_d, ["mr", "zf"], None, w.sigma2, w.p_total, prec)
    assert torch.equal(r.H, H_ref)
    for x, y in ((r.W, ref.W), (r.p_ant, ref.p_ant), (r.l21, ref.l21), (r.sinr, ref.sinr),
                 (r.rsum, ref.rsum), (r.info, ref.info)):
        assert torch.equal(x, y)
    Ho = _room_users(w)
    assert np.abs(host(r.H) - Ho).max() / np.abs(Ho).max() < 2e-6
    assert host(r.p_ant).sum(axis=(1, 2)) == pytest.approx([w.p_total, w.p_total], rel=1e-5)


def test_beamform_hall_zf_wide_path(D):
    # the hall's 32 users and 1024 APs (LoS, |h| ~ 1e-3) with the paper's
    # scaling at 10 dB targets, as the PA phase of bench.py forms it
    say("beamform ZF, hall deployment (wide path)")
    w = WL.hall_workload()
    H = c64(O.los_channel(w.user_xyz[0], w.ap_xyz[0], w.freq_hz)[None])
    r = _check_beamform(D, H, "zf", np.full(w.K, 10.0), w.sigma2, 0.0, "f32", 0.01, 1e-4)
    sinr_db = 10 * np.log10(host(r.sinr)[0])
    assert np.all(np.abs(sinr_db - 10.0) < 0.01)


def test_beamform_wide_singular_deployment_is_isolated(D):
    say("beamform ZF wide path, singular deployment")
    rng = np.random.default_rng(33)
    B, K, M = 3, 9, 600
    aps = np.stack([WL.uniform_positions(rng, M, 40, 40, 4.0) for _ in range(B)])
    users = np.stack([WL.uniform_positions(rng, K, 40, 40, 1.2) for _ in range(B)])
    users[1, 7] = users[1, 2]          # duplicate user in deployment 1
    Hc = np.stack([O.los_channel(users[b], aps[b], 3.5e9) for b in range(B)])
    H = c64(Hc)
    r = D.beamform(dev(H), "zf", None, 1e-12, 1.0, "f32")
    info = host(r.info)
    assert info[1] > 0 and info[[0, 2]].tolist() == [0, 0]
    assert not np.any(host(r.W)[1]) and not np.any(host(r.p_ant)[1])
    assert host(r.rsum)[1] == 0.0 and host(r.l21)[1] == 0.0 and not np.any(host(r.sinr)[1])
    Wr, sing = O.zf_precoder(H.astype(np.complex128), None, 1e-12, 1.0)
    assert sing[1] and not sing[[0, 2]].any()
    for b in (0, 2):
        assert np.linalg.norm(host(r.W)[b] - Wr[b]) / np.linalg.norm(Wr[b]) < 1e-4


def test_beamform_singular_deployment_is_isolated(D):
    say("beamform ZF singular deployment")
    rng = np.random.default_rng(31)
    B, K, M = 4, 4, 16
    aps = np.stack([WL.uniform_positions(rng, M, 20, 20, 4.0) for _ in range(B)])
    users = np.stack([WL.uniform_positions(rng, K, 20, 20, 1.2) for _ in range(B)])
    users[2, 3] = users[2, 1]          # duplicate user in deployment 2
    Hc = np.stack([O.los_channel(users[b], aps[b], 3.5e9) for b in range(B)])
    for prec in ("f64", "f32"):
        H = Hc if prec == "f64" else c64(Hc)
        r = D.beamform(dev(H), "zf", None, 1e-12, 1.0, prec)
        info = host(r.info)
        assert info[2] > 0 and info[[0, 1, 3]].tolist() == [0, 0, 0]
        W = host(r.W)
        assert not np.any(W[2]) and host(r.rsum)[2] == 0.0
        Wr, sing = O.zf_precoder(H.astype(np.complex128), None, 1e-12, 1.0)
        assert sing[2] and not sing[[0, 1, 3]].any()
        for b in (0, 1, 3):
            assert np.linalg.norm(W[b] - Wr[b]) / np.linalg.norm(Wr[b]) < 1e-4


# ---------------------------------------------------------------------------
# dmimo_powermap
# ---------------------------------------------------------------------------

def _check_map(D, aps, W, pts_desc, pts_xyz, f, sigma2, prec, tol_db, per_stream=True):
    Wd = dev(W)
    r = D.powermap(D.channel_params(f), dev(aps), Wd, pts_desc, sigma2, prec,
                   want_per_stream=per_stream)
    Hg = O.los_channel(pts_xyz, aps, f)
    Wc = W.astype(np.complex128)
    y_ref = O.power_map(Hg, Wc)
    check_db(host(r.power), y_ref, tol_db, what="power")
    if r.sinr is not None:
        s_ref, b_ref = O.sinr_map(Hg, Wc, sigma2)
        s = host(r.sinr)
        check_db(s, s_ref, tol_db, what="sinr")
        bk = host(r.best_k)
        P = np.abs(O.stream_fields(Hg, Wc)) ** 2
        top2 = np.sort(P, axis=1)[:, -2:] if P.shape[1] > 1 else None
        if top2 is not None:
            unique = top2[:, 1] > top2[:, 0] * (1 + 1e-4)
            np.testing.assert_array_equal(bk[unique], b_ref[unique])
            # elsewhere the chosen stream must be (numerically) a maximiser
            chosen = P[np.arange(len(bk)), bk]
            assert np.all(chosen >= top2[:, 1] * (1 - 1e-4))
        else:
            assert np.all(bk == 0)
    if per_stream:
        ps = host(r.per_stream)
        P = np.abs(O.stream_fields(Hg, Wc)) ** 2
        check_db(ps.ravel(), P.ravel(), tol_db, what="per-stream")
    return r


def test_powermap_focus_f64(D):
    say("powermap focus workload (M=16, K=1, 64x64, FP64)")
    w = WL.focus_workload()
    aps = w.ap_xyz[0]
    W = O.mr_precoder(O.los_channel(w.focal_xyz, aps, w.freq_hz), 1.0)
    _check_map(D, aps, W, D.grid_points(w.grid), grid_pts(w.grid), w.freq_hz, w.sigma2,
               "f64", 1e-9)


def test_powermap_focus_f32(D):
    say("powermap focus workload (M=16, K=1, 64x64, FP32)")
    w = WL.focus_workload()
    aps = w.ap_xyz[0]
    W = c64(O.mr_precoder(O.los_channel(w.focal_xyz, aps, w.freq_hz), 1.0))
    _check_map(D, aps, W, D.grid_points(w.grid), grid_pts(w.grid), w.freq_hz, w.sigma2,
               "f32", 0.01)


@pytest.mark.parametrize("prec", ["f32", "f16x3", "bf16x3"])
@pytest.mark.parametrize("precoder", ["mr", "zf"])
def test_powermap_room_small_grid(D, precoder, prec):
    say(f"powermap room {precoder} (M=64, K=8, 128x128 grid, {prec})")
    w = WL.room_workload(nx=128, ny=128)
    aps = w.ap_xyz[0]
    Hu = c64(_room_users(w))[0].astype(np.complex128)
    W = O.mr_precoder(Hu, 1.0) if precoder == "mr" else O.zf_precoder(Hu, None, w.sigma2, 1.0)[0]
    _check_map(D, aps, c64(W), D.grid_points(w.grid), grid_pts(w.grid), w.freq_hz, w.sigma2,
               prec, MAP_TOL[prec])


@pytest.mark.parametrize("precoder", ["mr", "zf"])
def test_powermap_room_full_grid_sampled_rows(D, precoder):
    # the full 512 x 512 launch, checked on 6 sampled rows against the oracle
    say(f"powermap room {precoder} full 512x512, sampled rows")
    w = WL.room_workload()
    aps = w.ap_xyz[0]
    Hu = c64(_room_users(w))[0].astype(np.complex128)
    W = c64(O.mr_precoder(Hu, 1.0) if precoder == "mr" else O.zf_precoder(Hu, None, w.sigma2, 1.0)[0])
    r = D.powermap(D.channel_params(w.freq_hz), dev(aps), dev(W), D.grid_points(w.grid),
                   w.sigma2, "f32")
    power = host(r.power).reshape(512, 512)
    sinr = host(r.sinr).reshape(512, 512)
    rows = [0, 1, 137, 255, 256, 511]
    pts = grid_pts(w.grid).reshape(512, 512, 3)[rows].reshape(-1, 3)
    Hg = O.los_channel(pts, aps, w.freq_hz)
    y_ref = O.power_map(Hg, W.astype(np.complex128))
    s_ref, _ = O.sinr_map(Hg, W.astype(np.complex128), w.sigma2)
    # floor taken relative to the full-map peak estimate from the sample
    check_db(power[rows].ravel(), y_ref, 0.01, what="power rows")
    check_db(sinr[rows].ravel(), s_ref, 0.01, what="sinr rows")
    assert np.all(np.isfinite(power)) and np.all(power > 0)


@pytest.mark.parametrize("prec", ["f32", "f16x3", "bf16x3"])
@pytest.mark.parametrize("K", [1, 2, 3, 5, 8, 12, 16, 32])
def test_powermap_stream_counts(D, K, prec):
    say(f"powermap K={K} list points (N=1000 ragged, M=48), {prec}")
    rng = np.random.default_rng(40 + K)
    M = 48
    aps = WL.uniform_positions(rng, M, 20, 20, 4.0)
    pts = WL.uniform_positions(rng, 1000, 20, 20, 1.2)
    W = c64(WL.complex_normal(rng, (K, M)) * 0.1)
    _check_map(D, aps, W, D.list_points(dev(pts), 1000), pts, 3.5e9, 1e-12, prec, MAP_TOL[prec])


@pytest.mark.parametrize("prec", ["f16x3", "bf16x3"])
def test_powermap_mixed_weight_dynamic_range(D, prec):
    # weights spanning 1e-6 .. 1e4 across 64-antenna chunks, M = 200 (4 chunks, ragged)
    say(f"powermap weights over 10 decades, M=200, K=4, {prec}")
    rng = np.random.default_rng(77)
    M, K = 200, 4
    aps = WL.uniform_positions(rng, M, 20, 20, 4.0)
    pts = WL.uniform_positions(rng, 700, 20, 20, 1.2)
    mag = 10.0 ** rng.uniform(-6, 4, size=(K, M))
    W = c64(WL.complex_normal(rng, (K, M)) * mag)
    _check_map(D, aps, W, D.list_points(dev(pts), 700), pts, 5.8e9, 1e-12, prec, MAP_TOL[prec])


def test_powermap_single_point_single_antenna(D):
    say("powermap N=1, M=1, K=1 (Friis)")
    aps = np.array([[0.0, 0.0, 3.0]])
    pts = np.array([[0.0, 0.0, 0.0]])
    f = 3.5e9
    W = c64(O.mr_precoder(O.los_channel(pts, aps, f), 1.0))
    r = D.powermap(D.channel_params(f), dev(aps), dev(W), D.list_points(dev(pts), 1), 1e-12,
                   "f32")
    assert host(r.power)[0] == pytest.approx(5.1624e-6, rel=1e-4)


# antennas in the map plane, some exactly on grid points (d = 0, the near-field
# clamp active) and some within d_min of a row: the FP32 row loop keeps its
# zero guard and clamp for those chunks (the guard-free loop runs only where
# every antenna of the chunk is more than d_min off the row); K = 8, M = 70
# (a ragged second chunk), against the oracle at every point
def test_powermap_antennas_in_the_map_plane(D):
    say("powermap: antennas in the map plane (guarded row loop), K=8, M=70")
    rng = np.random.default_rng(5)
    f = 3.5e9
    g = WL.Grid(0.0, 0.0, 0.25, 0.25, 1.2, 64, 64)        # points at (i + 0.5) / 4
    pts = grid_pts(g)
    M, K = 70, 8
    aps = WL.uniform_positions(rng, M, 16, 16, 4.0)
    on = rng.choice(64 * 64, 12, replace=False)
    aps[:12] = pts[on]                                    # on grid points, z = 1.2
    aps[12:20, 2] = 1.2 + rng.uniform(-0.005, 0.005, 8)   # within d_min of the plane
    users = WL.uniform_positions(rng, K, 16, 16, 1.2)
    W = c64(O.mr_precoder(O.los_channel(users, aps, f), 1.0))
    r = D.powermap(D.channel_params(f), dev(aps), dev(W), D.grid_points(g), 1e-12, "f32")
    power = host(r.power)
    assert np.all(np.isfinite(power)) and np.all(np.isfinite(host(r.sinr)))
    Hg = O.los_channel(pts, aps, f)
    Wc = W.astype(np.complex128)
    check_db(power, O.power_map(Hg, Wc), MAP_TOL["f32"], what="power")
    s_ref, _ = O.sinr_map(Hg, Wc, 1e-12)
    check_db(host(r.sinr), s_ref, MAP_TOL["f32"], what="sinr")


# The many-stream split-precision body (K > 8): a near-field clamp d_min ten
# times below lambda / (4 pi), so that |h| reaches 10 (the FP16 body scales h
# by 2^10 instead of 2^14), with antennas on grid points (d = 0) and within
# d_min of the map plane; a 100 x 23 grid, so that some workgroups span two
# rows (the general path) and the others lie on one row (guarded chunks next
# to the plane); M = 150 (a ragged third chunk).  Every point against the
# oracle with the same d_min.
@pytest.mark.parametrize("prec", ["f16x3", "bf16x3"])
@pytest.mark.parametrize("K", [9, 16, 24, 32])
def test_powermap_many_streams_small_dmin(D, K, prec):
    say(f"powermap K={K} M=150, d_min = lambda/(40 pi), antennas in the plane, {prec}")
    rng = np.random.default_rng(300 + K)
    f = 5.8e9
    lam = O.wavelength(f)
    d_min = lam / (40.0 * math.pi)
    g = WL.Grid(0.0, 0.0, 0.2, 0.2, 1.0, 100, 23)
    pts = grid_pts(g)
    M = 150
    aps = WL.uniform_positions(rng, M, 20, 4.6, 5.0)
    on = rng.choice(len(pts), 10, replace=False)
    aps[:10] = pts[on]                                     # on grid points
    aps[10:20, 2] = 1.0 + rng.uniform(-0.5, 0.5, 10) * d_min   # within d_min of the plane
    users = WL.uniform_positions(rng, K, 20, 4.6, 1.0)
    W = c64(O.mr_precoder(O.los_channel(users, aps, f, d_min=d_min), 1.0))
    r = D.powermap(D.channel_params(f, D.CH_LOS, 0.0, d_min), dev(aps), dev(W),
                   D.grid_points(g), 1e-12, prec)
    power = host(r.power)
    assert np.all(np.isfinite(power)) and np.all(np.isfinite(host(r.sinr)))
    Hg = O.los_channel(pts, aps, f, d_min=d_min)
    assert np.abs(Hg).max() > 8.0                          # the clamp bound, 10, is reached
    Wc = W.astype(np.complex128)
    check_db(power, O.power_map(Hg, Wc), MAP_TOL[prec], what="power")
    s_ref, _ = O.sinr_map(Hg, Wc, 1e-12)
    check_db(host(r.sinr), s_ref, MAP_TOL[prec], what="sinr")


# Weights of each stream spanning ten decades from chunk to chunk (M = 320,
# five chunks): the FP16 stream scales change between chunks and the
# accumulators are rescaled; K = 20 and 32 on a grid of rows far below the
# antennas (the guard-free row loop).
@pytest.mark.parametrize("prec", ["f16x3", "bf16x3"])
@pytest.mark.parametrize("K", [20, 32])
def test_powermap_many_streams_weight_dynamic_range(D, K, prec):
    say(f"powermap K={K} M=320, weights over 10 decades per stream, {prec}")
    rng = np.random.default_rng(500 + K)
    M, f = 320, 5.8e9
    aps = WL.uniform_positions(rng, M, 30, 30, 5.0)
    g = WL.Grid(0.0, 0.0, 30.0 / 256, 30.0 / 24, 1.0, 256, 24)
    mag = 10.0 ** (rng.uniform(-6, 4, size=(K, 1)) + rng.uniform(-3, 3, size=(1, M // 64)).repeat(64, 1))
    W = c64(WL.complex_normal(rng, (K, M)) * mag)
    _check_map(D, aps, W, D.grid_points(g), grid_pts(g), f, 1e-12, prec, MAP_TOL[prec],
               per_stream=True)


@pytest.mark.parametrize("prec", ["f32", "f16x3", "bf16x3"])
def test_powermap_hall_sampled(D, prec):
    # the full-size hall map (N = 2048^2, M = 1024, K = 32) in one launch,
    # checked on sampled rows
    say(f"powermap hall full 2048x2048, K=32, M=1024, {prec}, sampled rows")
    w = WL.hall_workload()
    aps = w.ap_xyz[0]
    Hu = c64(O.los_channel(w.user_xyz[0], aps, w.freq_hz)).astype(np.complex128)
    W = c64(O.zf_precoder(Hu, None, w.sigma2, 1.0)[0])
    r = D.powermap(D.channel_params(w.freq_hz), dev(aps), dev(W), D.grid_points(w.grid),
                   w.sigma2, prec)
    power = host(r.power).reshape(2048, 2048)
    sinr = host(r.sinr).reshape(2048, 2048)
    rows = [0, 1023, 2047]
    pts = grid_pts(w.grid).reshape(2048, 2048, 3)[rows].reshape(-1, 3)
    Hg = O.los_channel(pts, aps, w.freq_hz)
    Wc = W.astype(np.complex128)
    check_db(power[rows].ravel(), O.power_map(Hg, Wc), MAP_TOL[prec], what="power rows")
    s_ref, _ = O.sinr_map(Hg, Wc, w.sigma2)
    check_db(sinr[rows].ravel(), s_ref, MAP_TOL[prec], what="sinr rows")


def _same_maps_joint(prec, batch, one):
    # a joint launch (maps of K <= 8 streams with 8 < maps K <= 32, one
    # contraction of all their streams) against the single map: per-stream
    # powers, power and SINR within the precision's rounding, the best stream
    # equal wherever the two largest streams are not within that rounding
    import torch
    rtol = 2e-5 if prec == "f32" else 2e-4
    ps, po = batch.per_stream.double(), one.per_stream.double()
    scale = po.amax(dim=-1, keepdim=True)
    assert torch.all((ps - po).abs() <= rtol * scale)
    for a, b in ((batch.power, one.power), (batch.sinr, one.sinr)):
        assert torch.allclose(a.double(), b.double(), rtol=4 * rtol, atol=0.0)
    top2 = po.topk(2, dim=-1).values
    clear = (top2[..., 0] - top2[..., 1]) > 4 * rtol * top2[..., 0]
    assert torch.equal(batch.best_k[clear], one.best_k[clear])


# several precoders over the same points in one launch (map p on grid row p of
# the kernel) equal one call per precoder bit for bit, in every kernel family:
# FP32 VALU (K <= 2), FP32 MFMA (K <= 8, 16, 32), FP64, FP16x3, BF16x3; a
# ragged grid (41 x 29) and a ragged antenna chunk (M = 70).  Maps of K <= 8
# streams with 8 < maps K <= 32 in FP32 or the split modes run as one joint
# contraction of all their streams (each term synthesised once for all maps):
# there the maps equal the single calls to the rounding of the products
@pytest.mark.parametrize("prec,K,kind", [("f32", 2, "grid"), ("f32", 8, "grid"), ("f32", 12, "grid"),
                                         ("f32", 32, "grid"), ("f64", 8, "grid"), ("f16x3", 8, "grid"),
                                         ("bf16x3", 20, "grid"), ("f32", 8, "list"), ("f64", 3, "list"),
                                         ("bf16x3", 5, "grid"), ("f32", 3, "list")])
def test_powermap_batch_equals_single_maps(D, prec, K, kind):
    import torch
    say(f"powermap batch of 3 precoders, K={K}, {prec}, {kind} points")
    rng = np.random.default_rng(K + 7)
    M, P = 70, 3
    aps = WL.uniform_positions(rng, M, 20, 20, 3.0)
    g = WL.Grid(0.0, 0.0, 20 / 41, 20 / 29, 1.2, 41, 29)
    if kind == "grid":
        pts, n = D.grid_points(g), g.nx * g.ny
    else:
        xyz = dev(WL.uniform_positions(rng, 1000, 20, 20, 1.2)[None])
        pts, n = D.list_points(xyz, 1000), 1000
    Wn = WL.complex_normal(rng, (P, K, M)) * 0.05
    W = dev(Wn if prec == "f64" else c64(Wn))
    params = D.channel_params(3.5e9)
    apd = dev(aps)
    r = D.powermap_batch(params, apd, W, pts, 1e-9, prec, want_per_stream=True)
    assert tuple(r.power.shape) == (P, n)
    joint = prec != "f64" and K > 2 and K <= 8 and 8 < P * K <= 32
    for p in range(P):
        one = D.powermap(params, apd, W[p].contiguous(), pts, 1e-9, prec, want_per_stream=True)
        if joint:
            class Map:
                pass
            b = Map()
            b.power, b.sinr, b.best_k, b.per_stream = r.power[p], r.sinr[p], r.best_k[p], r.per_stream[p]
            _same_maps_joint(prec, b, one)
            continue
        for a, b in ((r.power[p], one.power), (r.sinr[p], one.sinr), (r.best_k[p], one.best_k),
                     (r.per_stream[p], one.per_stream)):
            assert torch.equal(a, b), p


# the bench step's two maps (MR and ZF of the room's 8 users, 512 x 512 grid)
# in one launch (one joint contraction of the 16 streams) equal the two single
# calls to the rounding of the products, and the oracle on sampled rows
@pytest.mark.parametrize("prec", ["f32", "f16x3"])
def test_powermap_batch_room_step_maps(D, prec):
    say(f"powermap batch: room MR + ZF maps, 512 x 512, {prec}")
    w = WL.room_workload()
    aps = w.ap_xyz[0]
    Hu = O.los_channel(w.user_xyz[0], aps, w.freq_hz)
    Wst = np.stack([O.mr_precoder(Hu[None], 1.0)[0], O.zf_precoder(Hu[None], None, w.sigma2, 1.0)[0][0]])
    W = dev(c64(Wst))
    params, apd, pts = D.channel_params(w.freq_hz), dev(aps), D.grid_points(w.grid)
    r = D.powermap_batch(params, apd, W, pts, w.sigma2, prec, want_per_stream=True)
    rows = [0, 255, 511]
    Hg = O.los_channel(grid_pts(w.grid).reshape(512, 512, 3)[rows].reshape(-1, 3), aps, w.freq_hz)
    for p in range(2):
        one = D.powermap(params, apd, W[p].contiguous(), pts, w.sigma2, prec, want_per_stream=True)

        class Map:
            pass
        b = Map()
        b.power, b.sinr, b.best_k, b.per_stream = r.power[p], r.sinr[p], r.best_k[p], r.per_stream[p]
        _same_maps_joint(prec, b, one)
        Wc = c64(Wst[p]).astype(np.complex128)
        check_db(host(r.power[p]).reshape(512, 512)[rows].ravel(), O.power_map(Hg, Wc),
                 MAP_TOL[prec], what=f"power rows, map {p}")
        check_db(host(r.sinr[p]).reshape(512, 512)[rows].ravel(), O.sinr_map(Hg, Wc, w.sigma2)[0],
                 MAP_TOL[prec], what=f"sinr rows, map {p}")


def test_room_steps_on_two_streams_equal_one_stream(D):
    # the benchmark's step (users' channels + MR/ZF in one launch, both maps in
    # one launch) with steps alternating over two streams, each with its own
    # outputs and no waits between them: every stream's outputs equal a
    # single-stream step bit for bit
    import torch
    say("room step on two streams (128 x 128 maps)")
    w = WL.room_workload(nx=128, ny=128)
    K, M, N = w.K, w.M, w.grid.n
    params = D.channel_params(w.freq_hz)
    ap_d, us_d, gpts = dev(w.ap_xyz), dev(w.user_xyz), D.grid_points(w.grid)
    ap0 = ap_d[0].contiguous()

    def step(out_pre, out_maps, stream):
        pre = D.beamform_users(params, ap_d, us_d, ("mr", "zf"), None, w.sigma2, w.p_total,
                               "f32", out=out_pre, stream=stream)
        maps = D.powermap_batch(params, ap0, pre.W.view(2, K, M), gpts, w.sigma2, "f32",
                                out=out_maps, stream=stream)
        return pre, maps

    ref_pre, ref_maps = step(None, None, None)
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = [step(None, None, s) for s in streams]
    torch.cuda.synchronize()
    for i in range(40):
        s = i % 2
        step(outs[s][0], outs[s][1], streams[s])
    torch.cuda.synchronize()
    for pre, maps in outs:
        assert torch.equal(pre.H, ref_pre.H) and torch.equal(pre.W, ref_pre.W)
        assert torch.equal(pre.sinr, ref_pre.sinr) and torch.equal(pre.p_ant, ref_pre.p_ant)
        for x, y in ((maps.power, ref_maps.power), (maps.sinr, ref_maps.sinr),
                     (maps.best_k, ref_maps.best_k)):
            assert torch.equal(x, y)
    assert tuple(ref_maps.power.shape) == (2, N)
