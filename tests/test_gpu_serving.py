"""GPU tests of the serving runtime (dmimo_server_*).

* A served query matches the FP64 oracle chain: users -> precoder -> map.
* A served query equals the one-shot calls (channel, beamform, powermap) bitwise.
* Each query's maps are bitwise the same alone and inside a mix of queries of
  different M, N, K, precoder and precision (continuous batching).
* Admission by HBM footprint: everything completes under a small budget, and
  a query that can never fit is refused with DMIMO_E_NOMEM.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import dberror  # noqa: E402
from oracle import dmimo_oracle as O  # noqa: E402
from oracle import pa_oracle as PA  # noqa: E402
from paper_2304_12745_amd import workloads as WL  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = {"f32": 0.01, "f16x3": 0.1, "bf16x3": 0.1}


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


def _room(rng, M, f):
    return WL.uniform_positions(rng, M, 20.0, 20.0, 4.0)


def _query_set(seed=5):
    """Deployments and a mix of query shapes (M, N, K, precoder, precision)."""
    rng = np.random.default_rng(seed)
    deps = [(16, 0.92e9), (64, 3.5e9), (256, 5.8e9)]
    aps = [_room(rng, M, f) for M, f in deps]
    shapes = [(64, 64), (96, 80), (160, 160), (33, 47)]
    qs = []
    for i in range(12):
        d = i % 3
        K = (1, 4, 16)[i % 3] if deps[d][0] >= 16 else 1
        nx, ny = shapes[i % 4]
        prec = ("f32", "f16x3", "bf16x3")[(i // 3) % 3]
        pc = "zf" if i % 2 else "mr"
        users = WL.uniform_positions(rng, K, 20.0, 20.0, 1.2)
        grid = WL.Grid(0.0, 0.0, 20.0 / nx, 20.0 / ny, 1.2, nx, ny)
        qs.append(dict(dep=d, K=K, users=users, grid=grid, prec=prec, pc=pc))
    return deps, aps, qs


def _submit(D, srv, dep_ids, q, sigma2=1e-12):
    N = q["grid"].n
    power = torch.empty(N, device="cuda")
    sinr = torch.empty(N, device="cuda")
    t = srv.submit(dep_ids[q["dep"]], q["users"], q["pc"], D.grid_points(q["grid"]), sigma2, 1.0,
                   q["prec"], power, sinr)
    return t, power, sinr


def test_served_query_matches_oracle(D):
    rng = np.random.default_rng(3)
    M, K, f = 64, 4, 3.5e9
    aps = _room(rng, M, f)
    users = WL.uniform_positions(rng, K, 20, 20, 1.2)
    g = WL.Grid(0.0, 0.0, 20 / 90, 20 / 70, 1.2, 90, 70)      # 6300 points: ragged tiles
    pts = O.grid_points(g.x0, g.y0, g.dx, g.dy, g.z, g.nx, g.ny)
    Hu = O.los_channel(users, aps, f)
    Hg = O.los_channel(pts, aps, f)
    with D.Server(256 << 20, 8) as srv:
        dep = srv.add_deployment(D.channel_params(f), aps)
        for pc in ("mr", "zf"):
            W = O.mr_precoder(Hu, 1.0) if pc == "mr" else O.zf_precoder(Hu, None, 1e-12, 1.0)[0]
            y_ref = O.power_map(Hg, W)
            s_ref, _ = O.sinr_map(Hg, W, 1e-12)
            for prec in ("f32", "f16x3", "bf16x3"):
                say(f"served {pc} {prec}")
                t, power, sinr = _submit(D, srv, [dep], dict(dep=0, K=K, users=users, grid=g,
                                                             prec=prec, pc=pc))
                assert srv.wait(t, 60.0) == D.Q_DONE
                sp = dberror.summary(power.cpu().numpy(), y_ref, TOL[prec])
                ss = dberror.summary(sinr.cpu().numpy(), s_ref, TOL[prec])
                say(f"    power max {sp['max_db']:.2e} dB, sinr max {ss['max_db']:.2e} dB")
                assert sp["n_fail"] == 0 and ss["n_fail"] == 0
                st, ts, td = srv.poll(t)
                assert st == D.Q_DONE and td >= ts > 0
                srv.release(t)


def test_served_equals_one_shot_calls(D):
    deps, aps, qs = _query_set(seed=11)
    with D.Server(512 << 20, 16) as srv:
        ids = [srv.add_deployment(D.channel_params(f), a) for (M, f), a in zip(deps, aps)]
        for q in qs[:6]:
            M, f = deps[q["dep"]]
            say(f"one-shot vs served: M={M} K={q['K']} N={q['grid'].n} {q['pc']} {q['prec']}")
            t, power, sinr = _submit(D, srv, ids, q)
            assert srv.wait(t, 60.0) == D.Q_DONE
            p = D.channel_params(f)
            ap = torch.from_numpy(aps[q["dep"]]).cuda()
            H = D.channel(p, ap[None].contiguous(), D.list_points(torch.from_numpy(q["users"]).cuda(), q["K"]),
                          prec="f32")
            r = D.beamform(H, q["pc"], None, 1e-12, 1.0, q["prec"], outputs=False)
            m = D.powermap(p, ap, r.W[0], D.grid_points(q["grid"]), 1e-12, q["prec"], want_best=False)
            torch.cuda.synchronize()
            assert torch.equal(m.power, power) and torch.equal(m.sinr, sinr)
            srv.release(t)


def test_alone_equals_mix(D):
    deps, aps, qs = _query_set(seed=7)
    with D.Server(1 << 30, 32) as srv:
        ids = [srv.add_deployment(D.channel_params(f), a) for (M, f), a in zip(deps, aps)]
        alone = []
        for q in qs:
            t, power, sinr = _submit(D, srv, ids, q)
            assert srv.wait(t, 60.0) == D.Q_DONE
            alone.append((power.cpu().numpy(), sinr.cpu().numpy()))
            srv.release(t)
        say(f"alone: {len(alone)} queries done")
        subs = [_submit(D, srv, ids, q) for q in qs]        # all in flight together
        for i, (t, power, sinr) in enumerate(subs):
            assert srv.wait(t, 120.0) == D.Q_DONE
            np.testing.assert_array_equal(power.cpu().numpy(), alone[i][0])
            np.testing.assert_array_equal(sinr.cpu().numpy(), alone[i][1])
            srv.release(t)
        st = srv.stats()
        say(f"mix: {st}")
        assert st["completed"] == 2 * len(qs)


def test_admission_by_footprint(D):
    rng = np.random.default_rng(9)
    M, f = 64, 3.5e9
    aps = _room(rng, M, f)
    g = WL.Grid(0.0, 0.0, 20 / 256, 20 / 256, 1.2, 256, 256)   # outputs 2 x 256 KiB
    with D.Server(4 << 20, 16) as srv:
        dep = srv.add_deployment(D.channel_params(f), aps)
        subs = []
        for i in range(10):
            users = WL.uniform_positions(rng, 4, 20, 20, 1.2)
            subs.append(_submit(D, srv, [dep], dict(dep=0, K=4, users=users, grid=g, prec="f32",
                                                    pc="zf")))
        for t, _, _ in subs:
            assert srv.wait(t, 60.0) == D.Q_DONE
            srv.release(t)
        # a query whose maps alone exceed the budget can never be admitted
        big = WL.Grid(0.0, 0.0, 20 / 1024, 20 / 1024, 1.2, 1024, 1024)
        with pytest.raises(D.DmimoError) as ei:
            _submit(D, srv, [dep], dict(dep=0, K=4, users=WL.uniform_positions(rng, 4, 20, 20, 1.2),
                                        grid=big, prec="f32", pc="mr"))
        assert ei.value.status == 8
        with pytest.raises(D.DmimoError) as ei:
            srv.poll(987654321)
        assert ei.value.status == 9
        assert srv.stats()["completed"] == 10


def test_pa_queries_equal_one_shot_and_mix(D):
    """DMIMO_PA queries (the PA-aware precoder, eq. optim1 by normalised PGD):
    their maps equal the one-shot chain channel -> dmimo_pa_precoder ->
    dmimo_powermap bitwise, alone and inside a mix with MR/ZF queries, and
    match the oracle chain."""
    rng = np.random.default_rng(13)
    deps = [(64, 3.5e9), (256, 5.8e9), (16, 0.92e9)]
    aps = [_room(rng, M, f) for M, f in deps]
    lams, er, gamma = [1 / 15] * 400, [1.0] * 400, 10.0
    pa_qs, other = [], []
    for i in range(6):
        d = i % 3
        K = (8, 16, 4)[d]
        nx, ny = ((64, 64), (96, 80), (33, 47))[d]
        grid = WL.Grid(0.0, 0.0, 20.0 / nx, 20.0 / ny, 1.2, nx, ny)
        users = WL.uniform_positions(rng, K, 20.0, 20.0, 1.2)
        pa_qs.append(dict(dep=d, K=K, users=users, grid=grid, prec=("f32", "f16x3")[i % 2], pc="pa"))
        other.append(dict(dep=d, K=K, users=users, grid=grid, prec="f32", pc=("mr", "zf")[i % 2]))
    with D.Server(1 << 30, 32) as srv:
        ids = [srv.add_deployment(D.channel_params(f), a) for (M, f), a in zip(deps, aps)]
        with pytest.raises(D.DmimoError):       # no schedule yet
            _submit(D, srv, ids, pa_qs[0])
        srv.set_pa_schedule(lams, er, gamma)
        with pytest.raises(D.DmimoError):       # set once
            srv.set_pa_schedule(lams, er, gamma)
        alone = []
        for q in pa_qs:
            M, f = deps[q["dep"]]
            say(f"PA query alone: M={M} K={q['K']} N={q['grid'].n} {q['prec']}")
            t, power, sinr = _submit(D, srv, ids, q)
            assert srv.wait(t, 60.0) == D.Q_DONE
            p = D.channel_params(f)
            ap = torch.from_numpy(aps[q["dep"]]).cuda()
            H = D.channel(p, ap[None].contiguous(),
                          D.list_points(torch.from_numpy(q["users"]).cuda(), q["K"]), prec="f32")
            r = D.pa_precoder(H, lams, er, [gamma] * q["K"], 1e-12)
            m = D.powermap(p, ap, r.W[0], D.grid_points(q["grid"]), 1e-12, q["prec"], want_best=False)
            torch.cuda.synchronize()
            assert torch.equal(m.power, power) and torch.equal(m.sinr, sinr)
            alone.append((power.cpu().numpy(), sinr.cpu().numpy()))
            srv.release(t)
            if q["prec"] == "f32" and q["K"] == 8:
                # oracle chain: oracle H -> oracle PA precoder -> oracle map
                g = q["grid"]
                Hu = O.los_channel(q["users"], aps[q["dep"]], f)
                Wo, _, _ = PA.pa_precoder(Hu[None], np.full(q["K"], gamma), 1e-12, lams, er)
                pts = O.grid_points(g.x0, g.y0, g.dx, g.dy, g.z, g.nx, g.ny)
                y = O.power_map(O.los_channel(pts, aps[q["dep"]], f), Wo[0])
                sp = dberror.summary(alone[-1][0], y, 0.01)
                say(f"    oracle chain: power max {sp['max_db']:.2e} dB")
                assert sp["n_fail"] == 0
        subs = [_submit(D, srv, ids, q) for pair in zip(pa_qs, other) for q in pair]
        for i, (t, power, sinr) in enumerate(subs):
            assert srv.wait(t, 120.0) == D.Q_DONE
            if i % 2 == 0:
                np.testing.assert_array_equal(power.cpu().numpy(), alone[i // 2][0])
                np.testing.assert_array_equal(sinr.cpu().numpy(), alone[i // 2][1])
            srv.release(t)


# ---------------------------------------------------------------------------
# failure paths: singular ZF, full queue, cancel, queue time-out, resident
# uploads between running queries
# ---------------------------------------------------------------------------

def _big_query(D, srv, dep, rng, side=1024, K=16, prec="f32"):
    users = WL.uniform_positions(rng, K, 20.0, 20.0, 1.2)
    g = WL.Grid(0.0, 0.0, 20.0 / side, 20.0 / side, 1.2, side, side)
    power = torch.full((g.n,), -1.0, device="cuda")
    t = srv.submit(dep, users, "zf", D.grid_points(g), 1e-12, 1.0, prec, power)
    return t, power


def _drain(srv, tickets, timeout=60.0):
    states = []
    for t in tickets:
        states.append(srv.wait(t, timeout))
    return states


def test_zf_query_with_duplicate_users_fails(D):
    # two users at one place make G singular: the query ends FAILED with the
    # pivot as its info word, and a regular query beside it is unaffected
    say("serving: ZF with duplicated users -> FAILED, neighbour DONE")
    rng = np.random.default_rng(21)
    aps = _room(rng, 64, 3.5e9)
    with D.Server(256 << 20, 8) as srv:
        dep = srv.add_deployment(D.channel_params(3.5e9), aps)
        g = WL.Grid(0.0, 0.0, 20 / 64, 20 / 64, 1.2, 64, 64)
        users = WL.uniform_positions(rng, 4, 20, 20, 1.2)
        bad = users.copy()
        bad[2] = bad[0]
        outs = []
        for u in (bad, users):
            p = torch.full((g.n,), -1.0, device="cuda")
            outs.append((srv.submit(dep, u, "zf", D.grid_points(g), 1e-12, 1.0, "f32", p), p))
        st = _drain(srv, [t for t, _ in outs])
        assert st == [D.Q_FAILED, D.Q_DONE]
        assert srv.query_info(outs[0][0]) == 3 and srv.query_info(outs[1][0]) == 0
        torch.cuda.synchronize()
        assert torch.all(outs[1][1] > 0)
        # the one-shot call reports the same pivot
        Hu = O.los_channel(bad, aps, 3.5e9).astype(np.complex64)
        r = D.beamform(torch.from_numpy(Hu[None]).cuda(), "zf", None, 1e-12, 1.0, "f32")
        assert int(r.info[0]) == 3


def test_full_pending_queue_is_busy(D):
    # one admitted query at a time and a pending queue of 64: a burst of 100
    # large queries (2048 x 2048 points, 512 APs, K = 16: milliseconds each),
    # with every input prepared before the burst so that the submissions take
    # microseconds, gets DMIMO_E_BUSY once 64 wait; every accepted query
    # completes
    say("serving: pending queue full -> DMIMO_E_BUSY")
    rng = np.random.default_rng(22)
    side, n = 2048, 100
    g = WL.Grid(0.0, 0.0, 20.0 / side, 20.0 / side, 1.2, side, side)
    pts = D.grid_points(g)
    users = [WL.uniform_positions(rng, 16, 20.0, 20.0, 1.2) for _ in range(n)]
    outs = [torch.full((g.n,), -1.0, device="cuda") for _ in range(n)]
    torch.cuda.synchronize()
    with D.Server(1 << 30, 1) as srv:
        dep = srv.add_deployment(D.channel_params(5.8e9), _room(rng, 512, 5.8e9))
        tickets, busy = [], 0
        for i in range(n):
            try:
                tickets.append(srv.submit(dep, users[i], "zf", pts, 1e-12, 1.0, "f32", outs[i]))
            except D.DmimoError as e:
                assert e.status == 7
                busy += 1
        say(f"    accepted {len(tickets)}, busy {busy}")
        assert busy > 0 and len(tickets) >= 64
        assert all(s == D.Q_DONE for s in _drain(srv, tickets, 300.0))


def test_cancel_a_queued_query(D):
    say("serving: cancel before admission")
    rng = np.random.default_rng(23)
    with D.Server(1 << 30, 1) as srv:
        dep = srv.add_deployment(D.channel_params(5.8e9), _room(rng, 512, 5.8e9))
        t0, p0 = _big_query(D, srv, dep, rng, side=2048)
        t1, p1 = _big_query(D, srv, dep, rng)
        t2, p2 = _big_query(D, srv, dep, rng)
        srv.cancel(t1)
        st = _drain(srv, [t0, t1, t2], 120.0)
        assert st == [D.Q_DONE, D.Q_CANCELLED, D.Q_DONE]
        torch.cuda.synchronize()
        assert torch.all(p1 == -1.0)                  # never written
        assert torch.all(p0 > 0) and torch.all(p2 > 0)
        with pytest.raises(D.DmimoError) as e:        # admitted and finished: not cancellable
            srv.cancel(t0)
        assert e.value.status == 7


def test_queue_timeout(D):
    # a 1 ms admission time-out with one query admitted at a time: the
    # queries behind a long one time out, their outputs untouched
    say("serving: queue time-out")
    rng = np.random.default_rng(24)
    with D.Server(1 << 30, 1) as srv:
        dep = srv.add_deployment(D.channel_params(5.8e9), _room(rng, 512, 5.8e9))
        srv.set_queue_timeout(1e-3)
        qs = [_big_query(D, srv, dep, rng, side=2048)] + [_big_query(D, srv, dep, rng)
                                                           for _ in range(5)]
        st = _drain(srv, [t for t, _ in qs], 120.0)
        say(f"    states {st}")
        assert st[0] == D.Q_DONE
        assert D.Q_TIMED_OUT in st[1:]
        torch.cuda.synchronize()
        for s, (_, p) in zip(st, qs):
            if s == D.Q_TIMED_OUT:
                assert torch.all(p == -1.0)
            else:
                assert s == D.Q_DONE and torch.all(p > 0)


def test_geometry_uploaded_between_running_queries(D):
    # Resident uploads come from the top of the arena.  Two large ZF queries
    # (K = 32, M = 4096: a few MiB of scratch each) run while deployments are
    # added; the arena is sized so that, had the geometry been placed between
    # their blocks, no free block would hold the third, larger query once they
    # finish.  It must be admitted and complete.
    say("serving: add_deployment between running queries, then a larger query")
    rng = np.random.default_rng(25)
    M = 4096
    sA = D.workspace_size(D.CALL_BEAMFORM_ZF, 1, 24, M, 0, "f32") + 2 * 24 * M * 8
    sC = D.workspace_size(D.CALL_BEAMFORM_ZF, 1, 32, M, 0, "f32") + 2 * 32 * M * 8
    geo = (M * 24 + 255) // 256 * 256
    side = 256
    maps = side * side * 4
    budget = 2 * (sA + 2048) + 3 * geo + sA // 2 + 2 * maps + (1 << 20)
    assert sC > sA and sC + maps + 3 * geo < budget
    aps = [_room(rng, M, 5.8e9) for _ in range(3)]
    with D.Server(budget, 4) as srv:
        dep = srv.add_deployment(D.channel_params(5.8e9), aps[0])
        ta, pa = _big_query(D, srv, dep, rng, side=side, K=24)
        srv.add_deployment(D.channel_params(5.8e9), aps[1])
        tb, pb = _big_query(D, srv, dep, rng, side=side, K=24)
        srv.add_deployment(D.channel_params(5.8e9), aps[2])
        tc, pc = _big_query(D, srv, dep, rng, side=side, K=32)
        st = _drain(srv, [ta, tb, tc], 60.0)
        assert st == [D.Q_DONE] * 3, st
        torch.cuda.synchronize()
        assert torch.all(pc > 0)
