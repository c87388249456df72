"""Seeded input generators: determinism, shapes and the layout rules."""
import numpy as np

from paper_2304_12745_amd import workloads as WL


def test_seeded_and_deterministic():
    a = WL.room_workload(seed=2, nx=8, ny=8)
    b = WL.room_workload(seed=2, nx=8, ny=8)
    np.testing.assert_array_equal(a.ap_xyz, b.ap_xyz)
    np.testing.assert_array_equal(a.user_xyz, b.user_xyz)
    c = WL.room_workload(seed=7, nx=8, ny=8)
    assert not np.array_equal(a.ap_xyz, c.ap_xyz)


def test_room_layout():
    w = WL.room_workload()
    assert w.ap_xyz.shape == (1, 64, 3) and w.user_xyz.shape == (1, 8, 3)
    aps = w.ap_xyz[0]
    # jittered 8x8 grid of pitch 2.5 m: every AP within a quarter pitch of its cell centre
    cx = (np.arange(8) + 0.5) * 2.5
    centres = np.stack(np.meshgrid(cx, cx, indexing="xy"), -1).reshape(-1, 2)
    assert np.max(np.abs(aps[:, :2] - centres)) <= 0.625
    assert np.all(aps[:, 2] == 4.0)
    assert np.all((w.user_xyz[0, :, :2] >= 0) & (w.user_xyz[0, :, :2] <= 20))
    assert w.grid.n == 512 * 512 and w.grid.dx == 20 / 512


def test_batched_and_paper_shapes():
    w = WL.batched_workload(B=4)
    assert w.ap_xyz.shape == (4, 256, 3) and w.user_xyz.shape == (4, 16, 3)
    assert w.nlos.shape == (4, 16, 256) and w.nlos.dtype == np.complex64
    assert abs(np.mean(np.abs(w.nlos) ** 2) - 1.0) < 0.05
    p = WL.paper_workload(B=10)
    assert p.H.shape == (10, 8, 64)
    np.testing.assert_allclose(p.gamma_lin, 10.0)


def test_hall_is_a_regular_grid():
    w = WL.hall_workload(nx=16, ny=16)
    aps = w.ap_xyz[0]
    assert aps.shape == (1024, 3)
    np.testing.assert_allclose(np.unique(aps[:, 0]), (np.arange(32) + 0.5) * 50 / 32)


def test_serving_stream():
    pool = WL.serving_pool()
    assert len(pool) == 4 * 3 * 8
    qs = WL.serving_queries(pool, 500)
    t = np.array([q.t_arrival for q in qs])
    assert np.all(np.diff(t) > 0)
    # Poisson at 2000/s: mean gap 0.5 ms
    assert abs(np.mean(np.diff(t)) - 5e-4) < 1e-4
    for q in qs:
        M, f, _ = pool[q.dep]
        assert M == q.M and f == q.freq_hz
        assert q.grid.n == q.side * q.side and q.user_xyz.shape == (q.K, 3)


def test_subgrid_rows():
    g = WL.Grid(0.0, 0.0, 0.5, 0.25, 1.0, 4, 8)
    s = g.rows(2, 5)
    assert s.ny == 3 and s.y0 == 0.5 and s.n == 12
