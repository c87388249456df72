"""GPU parity of the PA-aware precoder on distributed deployments
(dmimo_pa_precoder: eq. optim1 solved by normalised PGD, Sec. III-IV) against
the FP64 oracle.  FP32 on the GPU; the normalised iteration is non-expansive,
so W stays within 1e-4 relative of the oracle, SINR within 1e-3 dB."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import dmimo_oracle as O  # noqa: E402
from oracle import pa_oracle as PA  # noqa: E402
from oracle import pgd_oracle as P  # noqa: E402
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


def _rooms(n, K, seed, side=8, pitch=2.5):
    """n user draws in one jittered ceiling-grid room (the room workload's geometry)."""
    rng = np.random.default_rng(seed)
    aps = WL.ceiling_grid(side, side, pitch, 4.0, jitter_frac=0.25, rng=rng)
    room = side * pitch
    Hs = [O.los_channel(WL.uniform_positions(rng, K, room, room, 1.2), aps, 3.5e9) for _ in range(n)]
    return np.stack(Hs)


def _rel(a, b):
    return np.linalg.norm(a - b, axis=(-2, -1)) / np.linalg.norm(b, axis=(-2, -1))


def _compare(D, H, gamma, sigma2, lams, er, tol_w=1e-4):
    r = D.pa_precoder(torch.from_numpy(H.astype(np.complex64)).cuda(), lams, er, gamma, sigma2)
    torch.cuda.synchronize()
    Hc = H.astype(np.complex64).astype(np.complex128)
    W, s, L = PA.pa_precoder(Hc, gamma, sigma2, lams, er)
    e = _rel(r.W.cpu().numpy(), W)
    say(f"    W rel err max {e.max():.2e}")
    assert e.max() < tol_w
    pm = O.antenna_power(W)
    np.testing.assert_allclose(r.p_ant.cpu().numpy(), pm, rtol=0,
                               atol=2 * tol_w * pm.max(axis=-1, keepdims=True).max())
    np.testing.assert_allclose(r.l21.cpu().numpy(), O.l21_norm(W), rtol=tol_w)
    sinr = O.user_sinr(Hc, W, sigma2)
    db = np.abs(10 * np.log10(r.sinr.cpu().numpy() / sinr)).max()
    say(f"    SINR max dB err {db:.2e}")
    assert db < 1e-3
    np.testing.assert_allclose(r.rsum.cpu().numpy(), O.sum_rate(sinr), atol=1e-3)
    return r, W


def test_room_deployments_match_oracle(D):
    say("pa_precoder: 12 room draws, K=8, M=64, 300 layers, lambda 1/15")
    H = _rooms(12, 8, seed=21)
    _compare(D, H, np.full(8, 10.0), 1e-12, [1 / 15] * 300, [1.0] * 300)


def test_varying_schedule_and_targets(D):
    say("pa_precoder: ragged K=5, M=64 rooms, per-user targets, varying schedule")
    H = _rooms(6, 5, seed=22)
    rng = np.random.default_rng(3)
    gamma = 10 ** (rng.uniform(0.5, 1.5, 5))
    lams = rng.uniform(0.0, 0.5, 60)
    er = rng.uniform(0.5, 1.0, 60)
    _compare(D, H, gamma, 3e-13, lams, er)


def test_zero_lambda_gives_zf_in_deployment_units(D):
    say("pa_precoder lambda = 0, 3000 iterations -> ZF (paper scaling), -90 dBm noise")
    H = _rooms(4, 8, seed=23)
    gamma = np.full(8, 10.0)
    r = D.pa_precoder(torch.from_numpy(H.astype(np.complex64)).cuda(), [0.0] * 3000, [1.0] * 3000,
                      gamma, 1e-12)
    Wzf, _ = O.zf_precoder(H.astype(np.complex64).astype(np.complex128), gamma, 1e-12, 0.0)
    e = _rel(r.W.cpu().numpy(), Wzf)
    say(f"    W rel err vs ZF max {e.max():.2e}")
    assert e.max() < 2e-4
    assert np.abs(10 * np.log10(r.sinr.cpu().numpy()) - 10.0).max() < 2e-3


def test_converged_precoder_saves_power_and_switches_aps_off(D):
    say("pa_precoder 20000 iterations on 2 rooms: PCG >= 1, APs off as in the oracle")
    H = _rooms(2, 8, seed=24)
    gamma = np.full(8, 10.0)
    r = D.pa_precoder(torch.from_numpy(H.astype(np.complex64)).cuda(), [1 / 15] * 20000,
                      [1.0] * 20000, gamma, 1e-12)
    Hc = H.astype(np.complex64).astype(np.complex128)
    W, _, _ = PA.pa_precoder(Hc, gamma, 1e-12, [1 / 15] * 20000, [1.0] * 20000)
    Wzf, _ = O.zf_precoder(Hc, gamma, 1e-12, 0.0)
    pcg_g = O.l21_norm(Wzf) / r.l21.cpu().numpy()
    pcg_o = P.pcg(Wzf, W)
    off_g = (r.p_ant.cpu().numpy() == 0).sum(axis=1)
    off_o = (O.antenna_power(W) == 0).sum(axis=1)
    say(f"    PCG gpu {pcg_g} oracle {pcg_o}; APs off gpu {off_g} oracle {off_o}")
    assert np.all(pcg_g >= 1.0) and np.abs(pcg_g - pcg_o).max() < 1e-3
    assert np.all(off_g >= 10) and np.abs(off_g - off_o).max() <= 1


def test_valu_path_k16_m256(D):
    say("pa_precoder K=16, M=256 (16x16 ceiling grid), 80 layers")
    H = _rooms(3, 16, seed=25, side=16, pitch=1.25)
    _compare(D, H, np.full(16, 10.0), 1e-12, [0.1] * 80, [0.9] * 80)


def test_zero_channel_and_scale_covariance(D):
    say("pa_precoder: an all-zero channel, and H scaled by 1e3")
    H = _rooms(3, 8, seed=26)
    H[1] = 0.0
    gamma = np.full(8, 10.0)
    lams, er = [0.2] * 40, [1.0] * 40
    r = D.pa_precoder(torch.from_numpy(H.astype(np.complex64)).cuda(), lams, er, gamma, 1e-12)
    W = r.W.cpu().numpy()
    assert np.all(W[1] == 0) and np.all(np.isfinite(W))
    assert r.l21[1].item() == 0.0 and np.all(np.isfinite(r.rsum.cpu().numpy()))
    r2 = D.pa_precoder(torch.from_numpy((H * 1e3).astype(np.complex64)).cuda(), lams, er, gamma, 1e-12)
    e = _rel(r2.W.cpu().numpy()[[0, 2]] * 1e3, W[[0, 2]])
    assert e.max() < 1e-5


def _hall_like(n, K, M, seed):
    """n user draws on a regular ceiling grid of M APs (the hall workload's
    geometry, 5.8 GHz), a square grid of side sqrt(M)."""
    rng = np.random.default_rng(seed)
    side = int(round(np.sqrt(M)))
    pitch = 50.0 / side
    aps = WL.ceiling_grid(side, side, pitch, 5.0)[:M]
    room = side * pitch
    return np.stack([O.los_channel(WL.uniform_positions(rng, K, room, room, 1.0), aps, 5.8e9)
                     for _ in range(n)])


def test_slab_path_hall_deployment(D):
    say("pa_precoder slab path: hall K=32, M=1024, 120 layers")
    H = _hall_like(1, 32, 1024, seed=31)
    _compare(D, H, np.full(32, 10.0), 1e-12, [1 / 15] * 120, [1.0] * 120)


@pytest.mark.parametrize("B,K,M", [(3, 20, 64), (2, 12, 300), (2, 32, 130), (1, 17, 4096)])
def test_slab_path_shapes(D, B, K, M):
    say(f"pa_precoder slab path: B={B} K={K} M={M}")
    rng = np.random.default_rng(B * 1000 + K * 10 + M)
    if M == 4096:
        H = _hall_like(B, K, M, seed=K)
        lams, er = [0.1] * 8, [1.0] * 8
    else:
        side = int(np.ceil(np.sqrt(M)))
        aps = WL.ceiling_grid(side, side, 20.0 / side, 4.0, jitter_frac=0.25, rng=rng)[:M]
        H = np.stack([O.los_channel(WL.uniform_positions(rng, K, 20.0, 20.0, 1.2), aps, 3.5e9)
                      for _ in range(B)])
        lams = rng.uniform(0.0, 0.4, 30)
        er = rng.uniform(0.5, 1.0, 30)
    _compare(D, H, rng.uniform(3.0, 20.0, K), 1e-12, lams, er)


def test_slab_path_zero_lambda_gives_zf(D):
    say("pa_precoder slab path lambda = 0, 1500 iterations -> ZF, K=24 M=512")
    H = _hall_like(1, 24, 512, seed=33)
    gamma = np.full(24, 10.0)
    r = D.pa_precoder(torch.from_numpy(H.astype(np.complex64)).cuda(), [0.0] * 1500, [1.0] * 1500,
                      gamma, 1e-12)
    Hc = H.astype(np.complex64).astype(np.complex128)
    Wo, _, _ = PA.pa_precoder(Hc, gamma, 1e-12, [0.0] * 1500, [1.0] * 1500)
    Wzf, _ = O.zf_precoder(Hc, gamma, 1e-12, 0.0)
    e = _rel(r.W.cpu().numpy(), Wo)
    say(f"    W rel err vs oracle {e.max():.2e}, oracle vs ZF {_rel(Wo, Wzf).max():.2e}")
    assert e.max() < 2e-4


def test_bench_launch_configuration_1024_rooms_sampled(D):
    """The benchmark's batched launch (1024 deployments: 64 antennas per wave),
    checked on 12 sampled deployments."""
    say("pa_precoder: 1024 room draws in one launch, 300 iterations, sampled")
    H = _rooms(1024, 8, seed=27)
    gamma = np.full(8, 10.0)
    r = D.pa_precoder(torch.from_numpy(H.astype(np.complex64)).cuda(), [1 / 15] * 300,
                      [1.0] * 300, gamma, 1e-12)
    torch.cuda.synchronize()
    s = np.sort(np.random.default_rng(1).choice(1024, 12, replace=False))
    Hc = H[s].astype(np.complex64).astype(np.complex128)
    W, _, _ = PA.pa_precoder(Hc, gamma, 1e-12, [1 / 15] * 300, [1.0] * 300)
    e = _rel(r.W.cpu().numpy()[s], W)
    say(f"    W rel err max {e.max():.2e}")
    assert e.max() < 1e-4
    np.testing.assert_allclose(r.l21.cpu().numpy()[s], O.l21_norm(W), rtol=1e-4)


def test_bf16x3_room_deployments(D):
    say("pa_precoder BF16x3: 12 room draws, K=8, M=64, 300 layers")
    H = _rooms(12, 8, seed=21)
    r = D.pa_precoder(torch.from_numpy(H.astype(np.complex64)).cuda(), [1 / 15] * 300, [1.0] * 300,
                      np.full(8, 10.0), 1e-12, prec="bf16x3")
    Hc = H.astype(np.complex64).astype(np.complex128)
    W, _, _ = PA.pa_precoder(Hc, np.full(8, 10.0), 1e-12, [1 / 15] * 300, [1.0] * 300)
    e = _rel(r.W.cpu().numpy(), W)
    db = np.abs(10 * np.log10(r.sinr.cpu().numpy() / O.user_sinr(Hc, W, 1e-12))).max()
    say(f"    W rel err max {e.max():.2e}, SINR max dB err {db:.2e}")
    assert e.max() < 2e-3 and db < 0.01
