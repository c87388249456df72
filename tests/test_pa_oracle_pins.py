"""Pins of the PA-aware precoder oracle on distributed deployments (eq. optim1
solved by PGD, Sec. III-IV, on normalised channels)."""
import numpy as np

from oracle import dmimo_oracle as O
from oracle import pa_oracle as PA
from oracle import pgd_oracle as P
from paper_2304_12745_amd import workloads as WL


def _room_channels(n=3, seed=5):
    rng = np.random.default_rng(seed)
    w = WL.room_workload(nx=4, ny=4)
    Hs = []
    for _ in range(n):
        users = WL.uniform_positions(rng, 8, 20.0, 20.0, 1.2)
        Hs.append(O.los_channel(users, w.ap_xyz[0], w.freq_hz))
    return np.stack(Hs), w


def test_normalisation_is_rms_and_top_eigenvalue():
    H, _ = _room_channels()
    s, L = PA.normalisation(H)
    for b in range(len(H)):
        assert abs(s[b] - np.linalg.norm(H[b]) / np.sqrt(H[b].size)) < 1e-15 * s[b] * 10
        sv = np.linalg.svd(H[b] / s[b], compute_uv=False)
        assert abs(L[b] - sv[0] ** 2) < 1e-9 * L[b]


def test_zero_lambda_converges_to_zf_in_deployment_units():
    """With lambda = 0 PGD from H^* converges to the minimum-norm solution of the
    constraint, i.e. ZF with the paper's scaling, in the deployment's own units
    (noise -90 dBm): checks the normalisation, the step and the back-mapping."""
    H, w = _room_channels(2)
    gamma = np.full(8, 10.0)
    W, s, L = PA.pa_precoder(H, gamma, w.sigma2, [0.0] * 4000, [1.0] * 4000)
    Wzf, _ = O.zf_precoder(H, gamma, w.sigma2, 0.0)
    err = np.linalg.norm(W - Wzf, axis=(-2, -1)) / np.linalg.norm(Wzf, axis=(-2, -1))
    assert err.max() < 1e-6
    sinr = O.user_sinr(H, W, w.sigma2)
    assert np.max(np.abs(10 * np.log10(sinr) - 10.0)) < 1e-4


def test_converged_pa_precoder_consumes_no_more_than_zf():
    """At the optimum of lambda ||W||_{2,1} + f/2 the consumed power cannot exceed
    that of ZF, which is feasible with f = 0: PCG >= 1 (Sec. VI-B)."""
    H, w = _room_channels(2, seed=6)
    gamma = np.full(8, 10.0)
    W, _, _ = PA.pa_precoder(H, gamma, w.sigma2, [1 / 15] * 20000, [1.0] * 20000)
    Wzf, _ = O.zf_precoder(H, gamma, w.sigma2, 0.0)
    pcg = P.pcg(Wzf, W)
    assert np.all(pcg >= 1.0) and pcg.mean() > 1.1
    pm = O.antenna_power(W)
    assert np.all(np.sum(pm < 1e-12 * pm.max(axis=-1, keepdims=True), axis=-1) > 10)   # APs off


def test_scale_covariance():
    """Scaling H by c scales W by 1/c; scaling the noise power by c^2 scales W by c."""
    H, w = _room_channels(1, seed=7)
    gamma = np.full(8, 10.0)
    lams, er = [0.2] * 50, [0.9] * 50
    W, _, _ = PA.pa_precoder(H, gamma, w.sigma2, lams, er)
    W2, _, _ = PA.pa_precoder(H * 1e3, gamma, w.sigma2, lams, er)
    W3, _, _ = PA.pa_precoder(H, gamma, w.sigma2 * 4.0, lams, er)
    np.testing.assert_allclose(W2, W / 1e3, rtol=1e-11, atol=0)
    np.testing.assert_allclose(W3, W * 2.0, rtol=1e-11, atol=0)
