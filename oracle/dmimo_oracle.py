"""FP64 CPU oracle for the distributed-MIMO hot path.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark use this module; the library never calls it, and
it shares no code with the HIP path.

Every function here is the plain definition of one step, written in numpy
complex128 / float64 with no blocking, fusion or reordering, so that it can be
checked against the paper by eye.

Notation (paper, Sec. II-A): M transmit antennas, K single-antenna users.
The precoder is W in C^{K x M} and the transmitted vector is x = W^T s.  The
channel is H in C^{K x M}, and user k receives r = H x + noise.  A coherent
sum therefore multiplies h by w with *no* conjugate, and maximum-ratio
precoding is W = H^* (Sec. VI-C, initialisation of PGD).

Readings of passages where the paper is silent or ambiguous:

* The noise parameter sigma_nu is called a variance in Sec. II-A.  The ZF
  constraint of eq. (optim1) yields SINR_k = gamma_k only if sigma_nu is a
  standard deviation.  Here ``sigma2`` is the noise *power*, and the ZF
  constraint uses sqrt(sigma2).
* The SINR formula is not printed.  SINR_k = |A_kk|^2 /
  (sum_{j != k} |A_kj|^2 + sigma2) with A = H W^T, which follows from the
  signal model with unit-power, uncorrelated symbols.
* The paper is silent on geometry, carrier and path loss.  The channel between
  an antenna and a point follows the free-space spherical-wave model of the
  distributed-antenna workloads: amplitude lambda / (4 pi d) and phase
  -2 pi d / lambda.  A near-field clamp max(d, d_min) with d_min = lambda/(4 pi)
  keeps |h| <= 1; no workload reaches it.
* Rician fading (the batched workload) scales a CN(0,1) NLoS draw by the same
  path amplitude as the LoS term.
* Total-power scaling (MR and ZF at P watts) uses one common scalar per
  deployment, chosen so that ||W||_F^2 = P (eq. txpower).
* A power map is the total received signal power sum_k |z_k|^2 (streams are
  uncorrelated with unit power).  The SINR map takes the best stream,
  max_k SINR_k, with ties resolved to the lowest k.

Parity pins: every function in this module is pinned by the ``-m "not gpu"``
tests in tests/test_oracle_pins.py.  The pins are closed forms, special cases,
brute force and a value printed in the paper.
"""
from __future__ import annotations

import numpy as np

SPEED_OF_LIGHT = 299_792_458.0  # m/s


# ---------------------------------------------------------------------------
# geometry and channel
# ---------------------------------------------------------------------------

def wavelength(freq_hz: float) -> float:
    """Carrier wavelength lambda = c / f."""
    return SPEED_OF_LIGHT / float(freq_hz)


def grid_points(x0, y0, dx, dy, z, nx, ny) -> np.ndarray:
    """Cell centres of a regular evaluation grid, flat index n = j*nx + i.

    Point (i, j) = (x0 + (i+1/2) dx, y0 + (j+1/2) dy, z).  Returns [nx*ny][3].
    """
    i = np.arange(nx, dtype=np.float64)
    j = np.arange(ny, dtype=np.float64)
    xs = x0 + (i + 0.5) * dx
    ys = y0 + (j + 0.5) * dy
    X, Y = np.meshgrid(xs, ys, indexing="xy")   # [ny][nx]: x varies fastest
    pts = np.empty((ny * nx, 3), dtype=np.float64)
    pts[:, 0] = X.ravel()
    pts[:, 1] = Y.ravel()
    pts[:, 2] = z
    return pts


def distances(points: np.ndarray, aps: np.ndarray) -> np.ndarray:
    """Euclidean distance d[n, m] = ||p_n - a_m||_2 in FP64.  [N][3],[M][3] -> [N][M]."""
    diff = points[:, None, :] - aps[None, :, :]
    return np.sqrt(np.sum(diff * diff, axis=-1))


def default_d_min(freq_hz: float) -> float:
    """Near-field clamp distance lambda / (4 pi): there |h| would reach 1."""
    return wavelength(freq_hz) / (4.0 * np.pi)


def los_channel(points, aps, freq_hz, d_min=None) -> np.ndarray:
    """Free-space spherical-wave channel h[n, m] = lambda/(4 pi d) exp(-j 2 pi d / lambda).

    The phase uses numpy's complex exponential on the full phase 2 pi d/lambda
    (libm range reduction).  The amplitude uses max(d, d_min).  Returns [N][M]
    complex128.
    """
    lam = wavelength(freq_hz)
    if d_min is None or d_min <= 0.0:
        d_min = default_d_min(freq_hz)
    d = distances(np.asarray(points, np.float64), np.asarray(aps, np.float64))
    amp = lam / (4.0 * np.pi * np.maximum(d, d_min))
    return amp * np.exp(-2j * np.pi * d / lam)


def rician_channel(points, aps, freq_hz, kappa_lin, g, d_min=None) -> np.ndarray:
    """Rician channel: path amplitude times [sqrt(k/(1+k)) LoS phase + sqrt(1/(1+k)) g].

    ``g`` is the CN(0,1) NLoS draw [N][M].  kappa_lin = 0 gives pure scattering.
    """
    lam = wavelength(freq_hz)
    if d_min is None or d_min <= 0.0:
        d_min = default_d_min(freq_hz)
    d = distances(np.asarray(points, np.float64), np.asarray(aps, np.float64))
    amp = lam / (4.0 * np.pi * np.maximum(d, d_min))
    los = np.exp(-2j * np.pi * d / lam)
    k = float(kappa_lin)
    return amp * (np.sqrt(k / (1.0 + k)) * los
                  + np.sqrt(1.0 / (1.0 + k)) * np.asarray(g, np.complex128))


# ---------------------------------------------------------------------------
# Gram, precoders, power epilogues (Sec. II, III, VI)
# ---------------------------------------------------------------------------

def gram(H: np.ndarray) -> np.ndarray:
    """K x K Gram G = H H^H, per deployment.  [..][K][M] -> [..][K][K].

    The same non-zero eigenvalues as the M x M matrix H^T H^* whose largest
    eigenvalue bounds the PGD step (Sec. IV and V).
    """
    H = np.asarray(H, np.complex128)
    return H @ np.conj(np.swapaxes(H, -1, -2))


def mr_precoder(H, p_total: float) -> np.ndarray:
    """Maximum-ratio precoder W = c H^* (Sec. VI-C: W^(0) = H^*).

    p_total > 0: c = sqrt(P) / ||H||_F, so that ||W||_F^2 = P.  Otherwise c = 1.
    """
    H = np.asarray(H, np.complex128)
    W = np.conj(H)
    if p_total > 0.0:
        fro = np.sqrt(np.sum(np.abs(H) ** 2, axis=(-2, -1), keepdims=True))
        W = W * (np.sqrt(p_total) / fro)
    return W


def mr_phase_precoder(H, p_total: float) -> np.ndarray:
    """Equal-gain (phase-only) MR: w_km = a exp(-j angle(h_km)).

    a = sqrt(P / (K M)) when p_total > 0, otherwise a = 1.
    """
    H = np.asarray(H, np.complex128)
    K, M = H.shape[-2], H.shape[-1]
    a = np.sqrt(p_total / (K * M)) if p_total > 0.0 else 1.0
    return a * np.exp(-1j * np.angle(H))


def zf_precoder(H, gamma_lin=None, sigma2: float = 1.0, p_total: float = 0.0):
    """Zero-forcing precoder (eq. optim1 constraint H W^T = sigma D_gamma^{1/2}).

    X = G^{-1} H is computed with an LU solve, not a Cholesky, and W ∝ conj(X).
    * p_total <= 0 (paper scaling): W = sqrt(sigma2) diag(sqrt(gamma)) conj(X),
      which meets the constraint exactly.
    * p_total > 0: W = c conj(X) with c chosen so that ||W||_F^2 = P
      (eq. txpower).  This gives every user the same SINR.

    Returns (W, singular), where ``singular`` flags deployments with
    cond(G) > 1e12.  W is zero there.
    """
    H = np.asarray(H, np.complex128)
    squeeze = H.ndim == 2
    if squeeze:
        H = H[None]
    B, K, M = H.shape
    G = gram(H)
    W = np.zeros_like(H)
    singular = np.zeros(B, dtype=bool)
    for b in range(B):
        if np.linalg.cond(G[b]) > 1e12:
            singular[b] = True
            continue
        X = np.linalg.solve(G[b], H[b])
        if p_total > 0.0:
            c = np.sqrt(p_total / np.sum(np.abs(X) ** 2))
            W[b] = c * np.conj(X)
        else:
            g = np.ones(K) if gamma_lin is None else np.asarray(gamma_lin, np.float64)
            W[b] = np.sqrt(sigma2) * np.sqrt(g)[:, None] * np.conj(X)
    if squeeze:
        return W[0], singular[0]
    return W, singular


def antenna_power(W) -> np.ndarray:
    """Per-antenna transmit power p_m = sum_k |w_km|^2 (Sec. II-B).  [..][K][M] -> [..][M]."""
    return np.sum(np.abs(np.asarray(W, np.complex128)) ** 2, axis=-2)


def tx_power(W) -> np.ndarray:
    """Total transmit power p_tx = ||W||_F^2 (eq. txpower)."""
    return np.sum(np.abs(np.asarray(W, np.complex128)) ** 2, axis=(-2, -1))


def l21_norm(W) -> np.ndarray:
    """||W||_{2,1} = sum_m sqrt(p_m).  The PA consumed power is alpha ||W||_{2,1} (eq. effmodel)."""
    return np.sum(np.sqrt(antenna_power(W)), axis=-1)


def user_gains(H, W) -> np.ndarray:
    """Effective gains A = H W^T: user k receives stream j with gain A_kj (Sec. II-A)."""
    H = np.asarray(H, np.complex128)
    W = np.asarray(W, np.complex128)
    return H @ np.swapaxes(W, -1, -2)


def user_sinr(H, W, sigma2: float) -> np.ndarray:
    """SINR_k = |A_kk|^2 / (sum_{j != k} |A_kj|^2 + sigma2), with A = H W^T.  [..][K]."""
    A = user_gains(H, W)
    P = np.abs(A) ** 2
    K = P.shape[-1]
    eye = np.eye(K, dtype=bool)
    signal = np.sum(np.where(eye, P, 0.0), axis=-1)
    interference = np.sum(np.where(eye, 0.0, P), axis=-1)
    return signal / (interference + sigma2)


def sum_rate(sinr) -> np.ndarray:
    """R_sum = sum_k log2(1 + SINR_k) (Sec. VI-B)."""
    return np.sum(np.log2(1.0 + np.asarray(sinr, np.float64)), axis=-1)


# ---------------------------------------------------------------------------
# maps: coherent sums at evaluation points
# ---------------------------------------------------------------------------

def stream_fields(Hpts, W) -> np.ndarray:
    """z_k[n] = sum_m h[n, m] w_km (no conjugate: x = W^T s).  [N][M],[K][M] -> [N][K]."""
    return np.asarray(Hpts, np.complex128) @ np.asarray(W, np.complex128).T


def power_map(Hpts, W) -> np.ndarray:
    """Received signal power y[n] = sum_k |z_k[n]|^2.  For K = 1 this is |sum_m h w|^2."""
    Z = stream_fields(Hpts, W)
    return np.sum(np.abs(Z) ** 2, axis=-1)


def sinr_map(Hpts, W, sigma2: float):
    """Best-stream SINR map and the chosen stream.

    SINR[n] = max_k |z_k|^2 / (sum_{j != k} |z_j|^2 + sigma2).  The argmax is
    also the stream of largest |z_k|^2 (SINR_k increases with |z_k|^2).  Ties
    go to the lowest k.  Returns (sinr [N], best_k [N] int32).
    """
    Z = stream_fields(Hpts, W)
    P = np.abs(Z) ** 2
    N, K = P.shape
    sinr = np.empty((N, K))
    for k in range(K):
        others = np.delete(P, k, axis=1).sum(axis=1) if K > 1 else np.zeros(N)
        sinr[:, k] = P[:, k] / (others + sigma2)
    best = np.argmax(sinr, axis=1).astype(np.int32)
    return sinr[np.arange(N), best], best
