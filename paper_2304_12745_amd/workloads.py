"""Seeded synthetic inputs for the distributed-MIMO hot path.

This module only draws random numbers and lays out geometry: antenna and user
positions, evaluation-grid descriptors, Rayleigh / NLoS draws and the serving
query stream.  It holds none of the method's arithmetic (no distance, channel,
Gram, precoder or power computation), so that the HIP path and the FP64 oracle
can both take their inputs from here without sharing any of the computation.

Every generator takes an explicit seed and uses ``numpy.random.default_rng``.
Within one workload the draw order is fixed: access points, then users, then
the focal point, then NLoS entries, then the query stream.

Workloads (sizes as used by the tests and the benchmark):

* ``paper``  - the paper's own setting (Sec. VI-A, VI-C): i.i.d. Rayleigh
  channels ``[H]_{k,m} ~ CN(0,1)``, K=8 users, M=64 antennas, per-user SINR
  target 10 dB, noise standard deviation 1, a test set of 5000 channels.
* ``focus``  - M=16 APs uniform on the ceiling (z=3 m) of a 10x10x3 m room,
  920 MHz, MR focused on one seeded point at z=1 m, 64x64 map at z=1 m, FP64.
* ``room``   - M=64 APs on a jittered 8x8 ceiling grid (pitch 2.5 m, z=4 m)
  of a 20x20x4 m room, 3.5 GHz, K=8 users at z=1.2 m, MR and ZF at 1 W,
  noise -90 dBm, 512x512 power/SINR maps at z=1.2 m.
* ``batched`` - 1024 independent 20x20x4 m rooms, each with M=256 APs on a
  jittered 16x16 ceiling grid (pitch 1.25 m), K=16 users at z=1.2 m, 5.8 GHz,
  Rician fading with K-factor 6 dB (CN(0,1) NLoS entries), ZF at 1 W.
* ``serving`` - Poisson stream of power-map queries of mixed sizes.
* ``hall``   - M=1024 APs on a regular 32x32 ceiling grid (pitch 1.5625 m,
  z=5 m) of a 50x50x5 m hall, 5.8 GHz, K=32 users at z=1 m, ZF at 1 W,
  2048x2048 map at z=1 m.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

NOISE_MINUS_90_DBM_W = 1e-12  # -90 dBm expressed in watts


@dataclass(frozen=True)
class Grid:
    """Regular evaluation grid: cell centres of an nx x ny tiling at height z.

    Point (i, j) sits at (x0 + (i + 1/2) dx, y0 + (j + 1/2) dy, z) and is stored
    at flat index n = j * nx + i.
    """
    x0: float
    y0: float
    dx: float
    dy: float
    z: float
    nx: int
    ny: int

    @property
    def n(self) -> int:
        return self.nx * self.ny

    def rows(self, j0: int, j1: int) -> "Grid":
        """The sub-grid made of rows j0 <= j < j1 (same points, same order)."""
        return Grid(self.x0, self.y0 + j0 * self.dy, self.dx, self.dy, self.z,
                    self.nx, j1 - j0)


@dataclass
class Workload:
    name: str
    freq_hz: float
    ap_xyz: np.ndarray                 # float64 [B][M][3]
    user_xyz: Optional[np.ndarray]     # float64 [B][K][3]
    grid: Optional[Grid] = None
    focal_xyz: Optional[np.ndarray] = None   # float64 [1][3]
    nlos: Optional[np.ndarray] = None        # complex64 [B][K][M]
    kappa_lin: float = 0.0                    # Rician K-factor (linear); 0 -> LoS
    sigma2: float = NOISE_MINUS_90_DBM_W     # noise power (W)
    p_total: float = 1.0                      # total transmit power (W)
    gamma_lin: Optional[np.ndarray] = None   # per-user SINR targets (linear)
    precoders: tuple = ("mr", "zf")
    H: Optional[np.ndarray] = None            # given channels (Rayleigh workload)
    extra: dict = field(default_factory=dict)

    @property
    def B(self) -> int:
        return self.ap_xyz.shape[0] if self.ap_xyz is not None else self.H.shape[0]

    @property
    def M(self) -> int:
        return self.ap_xyz.shape[1] if self.ap_xyz is not None else self.H.shape[2]

    @property
    def K(self) -> int:
        if self.user_xyz is not None:
            return self.user_xyz.shape[1]
        return self.H.shape[1]


# ---------------------------------------------------------------------------
# layout helpers (positions only)
# ---------------------------------------------------------------------------

def uniform_positions(rng, count, xmax, ymax, z):
    """``count`` points uniform over [0,xmax]x[0,ymax] at height z."""
    xy = rng.uniform(0.0, 1.0, size=(count, 2)) * np.array([xmax, ymax])
    return np.concatenate([xy, np.full((count, 1), float(z))], axis=1)


def ceiling_grid(nx, ny, pitch, z, jitter_frac=0.0, rng=None):
    """Cell centres of an nx x ny grid of the given pitch at height z.

    With ``jitter_frac`` > 0 every centre moves by U(-jitter_frac, jitter_frac)
    times the pitch in x and in y (independently).  Ordering: x fastest.
    """
    i = np.arange(nx)
    j = np.arange(ny)
    xs, ys = np.meshgrid((i + 0.5) * pitch, (j + 0.5) * pitch, indexing="xy")
    xy = np.stack([xs.ravel(), ys.ravel()], axis=1)
    if jitter_frac > 0.0:
        xy = xy + rng.uniform(-jitter_frac, jitter_frac, size=xy.shape) * pitch
    return np.concatenate([xy, np.full((nx * ny, 1), float(z))], axis=1)


def complex_normal(rng, shape, dtype=np.complex128):
    """CN(0,1) draws: real and imaginary parts N(0, 1/2), real part drawn first."""
    re = rng.standard_normal(size=shape)
    im = rng.standard_normal(size=shape)
    return ((re + 1j * im) / np.sqrt(2.0)).astype(dtype)


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

def paper_workload(seed=0, B=5000, K=8, M=64, gamma_db=10.0, sigma=1.0,
                   dtype=np.complex128):
    """The paper's Rayleigh test setting (Sec. VI-A and VI-C)."""
    rng = np.random.default_rng(seed)
    H = complex_normal(rng, (B, K, M), dtype)
    gamma = np.full(K, 10.0 ** (gamma_db / 10.0))
    return Workload(name="paper", freq_hz=0.0, ap_xyz=None, user_xyz=None,
                    H=H, sigma2=sigma * sigma, p_total=0.0, gamma_lin=gamma,
                    precoders=("mr", "zf"))


@dataclass
class UfpgdDatasets:
    train: np.ndarray     # complex64 [n_train][K][M]
    val: np.ndarray
    test: np.ndarray
    gamma_lin: np.ndarray
    sigma2: float


def ufpgd_datasets(n_train=100000, n_val=5000, n_test=5000, K=8, M=64, gamma_db=10.0, seed=0):
    """Training, validation and test channels of the paper's unfolding
    experiment (Sec. VI-A): independent Rayleigh draws H ~ CN(0, 1), drawn
    in that order from one seeded generator."""
    rng = np.random.default_rng(1000 + seed)
    tr = complex_normal(rng, (n_train, K, M), np.complex64)
    va = complex_normal(rng, (n_val, K, M), np.complex64)
    te = complex_normal(rng, (n_test, K, M), np.complex64)
    return UfpgdDatasets(tr, va, te, np.full(K, 10.0 ** (gamma_db / 10.0)), 1.0)


def focus_workload(seed=1, M=16, nx=64, ny=64):
    """Single-room MR focusing map at 920 MHz, computed in FP64."""
    rng = np.random.default_rng(seed)
    aps = uniform_positions(rng, M, 10.0, 10.0, 3.0)
    focal = uniform_positions(rng, 1, 10.0, 10.0, 1.0)
    grid = Grid(0.0, 0.0, 10.0 / nx, 10.0 / ny, 1.0, nx, ny)
    return Workload(name="focus", freq_hz=0.92e9, ap_xyz=aps[None],
                    user_xyz=focal[None], focal_xyz=focal, grid=grid,
                    p_total=1.0, precoders=("mr",))


def room_workload(seed=2, K=8, nx=512, ny=512):
    """20x20x4 m room, jittered 8x8 ceiling grid, 3.5 GHz, K users, MR and ZF."""
    rng = np.random.default_rng(seed)
    aps = ceiling_grid(8, 8, 2.5, 4.0, jitter_frac=0.25, rng=rng)
    users = uniform_positions(rng, K, 20.0, 20.0, 1.2)
    grid = Grid(0.0, 0.0, 20.0 / nx, 20.0 / ny, 1.2, nx, ny)
    return Workload(name="room", freq_hz=3.5e9, ap_xyz=aps[None],
                    user_xyz=users[None], grid=grid, p_total=1.0,
                    precoders=("mr", "zf"))


def batched_workload(seed=3, B=1024, K=16, side=16, pitch=1.25,
                     kappa_db=6.0):
    """B independent Rician rooms at 5.8 GHz, ZF at 1 W per deployment."""
    rng = np.random.default_rng(seed)
    M = side * side
    aps = np.stack([ceiling_grid(side, side, pitch, 4.0, jitter_frac=0.25,
                                 rng=rng) for _ in range(B)])
    room = side * pitch
    users = np.stack([uniform_positions(rng, K, room, room, 1.2)
                      for _ in range(B)])
    nlos = complex_normal(rng, (B, K, M), np.complex64)
    return Workload(name="batched", freq_hz=5.8e9, ap_xyz=aps,
                    user_xyz=users, nlos=nlos,
                    kappa_lin=10.0 ** (kappa_db / 10.0), p_total=1.0,
                    precoders=("zf",))


def hall_workload(seed=5, K=32, nx=2048, ny=2048):
    """50x50x5 m hall, regular 32x32 ceiling grid, 5.8 GHz, K=32 ZF users."""
    rng = np.random.default_rng(seed)
    aps = ceiling_grid(32, 32, 50.0 / 32, 5.0)
    users = uniform_positions(rng, K, 50.0, 50.0, 1.0)
    grid = Grid(0.0, 0.0, 50.0 / nx, 50.0 / ny, 1.0, nx, ny)
    return Workload(name="hall", freq_hz=5.8e9, ap_xyz=aps[None],
                    user_xyz=users[None], grid=grid, p_total=1.0,
                    precoders=("zf",))


# ---------------------------------------------------------------------------
# serving: deployment pool and Poisson query stream
# ---------------------------------------------------------------------------

SERVE_M = (16, 64, 256, 512)
SERVE_SIDE = (64, 256, 1024)           # grid is side x side points
SERVE_K = (1, 4, 16)
SERVE_F = (0.92e9, 3.5e9, 5.8e9)


@dataclass
class Query:
    t_arrival: float        # seconds from the start of the stream
    dep: int                # index into the deployment pool
    M: int
    K: int
    freq_hz: float
    side: int
    precoder: str           # "mr" or "zf"
    user_xyz: np.ndarray    # float64 [K][3]
    grid: Grid


def serving_pool(seed=4, per_combo=8):
    """Deployment pool: for every (M, f), ``per_combo`` rooms with APs uniform
    over a 20x20 m ceiling at z=4 m.  Returns a list of (M, f, ap_xyz)."""
    rng = np.random.default_rng(seed)
    pool = []
    for M in SERVE_M:
        for f in SERVE_F:
            for _ in range(per_combo):
                pool.append((M, f, uniform_positions(rng, M, 20.0, 20.0, 4.0)))
    return pool


def serving_queries(pool, n_queries, rate_hz=2000.0, seed=4):
    """Poisson stream of power-map queries over the pool (draw order: arrival
    gap, size choices, deployment, users)."""
    rng = np.random.default_rng(seed + 1000)
    t = 0.0
    out: List[Query] = []
    by_key = {}
    for idx, (M, f, _) in enumerate(pool):
        by_key.setdefault((M, f), []).append(idx)
    for _ in range(n_queries):
        t += rng.exponential(1.0 / rate_hz)
        M = int(rng.choice(SERVE_M))
        side = int(rng.choice(SERVE_SIDE))
        K = int(rng.choice(SERVE_K))
        f = float(rng.choice(SERVE_F))
        cands = by_key[(M, f)]
        dep = int(cands[rng.integers(len(cands))])
        users = uniform_positions(rng, K, 20.0, 20.0, 1.2)
        prec = "zf" if rng.uniform() < 0.5 else "mr"
        if K > M:
            prec = "mr"
        grid = Grid(0.0, 0.0, 20.0 / side, 20.0 / side, 1.2, side, side)
        out.append(Query(t, dep, M, K, f, side, prec, users, grid))
    return out
