"""Pins of the PGD / unfolded-PGD oracle (oracle/pgd_oracle.py).

* the prox is the Moreau minimiser of t||x|| + ||x - v||^2 / 2 (numerical
  optimisation, not the closed form);
* the step direction is the Wirtinger gradient (finite differences);
* lambda = 0 from W(0) = H^* converges to the ZF precoder (closed form);
* the objective f/2 + lambda ||W||_{2,1} decreases monotonically for eta <= 1/L;
* the limit satisfies the group-lasso optimality conditions;
* the statistics printed in the paper (tests/golden/paper_pgd_pcg.txt).
"""
import os

import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import dmimo_oracle as O
from oracle import pgd_oracle as P
from paper_2304_12745_amd import workloads as WL

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    out = {}
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split()
            out[k] = float(v)
    return out


def test_prox_is_the_moreau_minimiser():
    rng = np.random.default_rng(1)
    for t in (0.1, 0.7, 3.0):
        V = WL.complex_normal(rng, (3, 4))
        X = P.prox_l21(V, t)
        for m in range(4):
            v = np.concatenate([V[:, m].real, V[:, m].imag])

            def obj(x):
                return t * np.linalg.norm(x) + 0.5 * np.sum((x - v) ** 2)
            best = min((minimize(obj, x0, method="Nelder-Mead",
                                 options={"xatol": 1e-10, "fatol": 1e-14, "maxiter": 20000})
                        for x0 in (v, 0.5 * v, np.full(6, 1e-3))), key=lambda r: r.fun)
            x = np.concatenate([X[:, m].real, X[:, m].imag])
            assert obj(x) <= best.fun + 1e-9
            assert np.linalg.norm(x - best.x) < 1e-4
    # closed-form cases: below the threshold a column vanishes, above it the norm drops by t
    V = np.array([[3.0 + 4j], [0.0]])
    np.testing.assert_allclose(np.linalg.norm(P.prox_l21(V, 1.0)), 4.0)
    assert not np.any(P.prox_l21(V, 5.0))
    assert not np.any(P.prox_l21(V, 6.0))


def test_step_direction_is_the_wirtinger_gradient():
    rng = np.random.default_rng(2)
    H = WL.complex_normal(rng, (3, 5))
    W = WL.complex_normal(rng, (3, 5))
    gamma, sigma = np.array([1.0, 2.0, 5.0]), 0.7
    g = P.wirtinger_gradient(H, W, gamma, sigma)
    eps = 1e-6
    num = np.zeros_like(W)
    for k in range(3):
        for m in range(5):
            E = np.zeros_like(W)
            E[k, m] = eps
            dre = (P.smooth_term(H, W + E, gamma, sigma) - P.smooth_term(H, W - E, gamma, sigma)) / (2 * eps)
            dim = (P.smooth_term(H, W + 1j * E, gamma, sigma) - P.smooth_term(H, W - 1j * E, gamma, sigma)) / (2 * eps)
            num[k, m] = 0.5 * (dre + 1j * dim)       # d/dW^* = (d/dRe + j d/dIm) / 2
    np.testing.assert_allclose(g, num, rtol=1e-6, atol=1e-7)


def test_lambda_zero_converges_to_zf():
    w = WL.paper_workload(seed=3, B=4)
    L = np.linalg.eigvalsh(O.gram(w.H))[:, -1].max()
    W = P.pgd(w.H, w.gamma_lin, 1.0, 0.0, 1.0 / L, 400)
    Wzf, _ = O.zf_precoder(w.H, w.gamma_lin, 1.0, 0.0)
    np.testing.assert_allclose(W, Wzf, rtol=1e-8, atol=1e-10)


def test_objective_decreases_monotonically():
    w = WL.paper_workload(seed=4, B=3)
    lam = 1 / 15
    L = np.linalg.eigvalsh(O.gram(w.H))[:, -1].max()
    _, hist = P.pgd(w.H, w.gamma_lin, 1.0, lam, 1.0 / L, 200, history=True)
    F = np.array([P.smooth_term(w.H, W, w.gamma_lin, 1.0) / 2 + lam * O.l21_norm(W) for W in hist])
    assert np.all(np.diff(F, axis=0) <= 1e-12 * np.abs(F[:-1]))


def test_limit_satisfies_group_lasso_optimality():
    # PGD converges slowly (the paper's point): 40000 iterations on one channel
    w = WL.paper_workload(seed=5, B=1)
    lam = 0.3
    L = np.linalg.eigvalsh(O.gram(w.H))[:, -1].max()
    W = P.pgd(w.H, w.gamma_lin, 1.0, lam, 1.0 / L, 40000)
    G = P.wirtinger_gradient(w.H, W, w.gamma_lin, 1.0)
    norms = np.linalg.norm(W, axis=-2)
    for b in range(1):
        active = norms[b] > 1e-8
        assert active.any() and (~active).any()      # a sparse solution: some antennas are off
        r = G[b][:, active] + lam * W[b][:, active] / norms[b][active]
        assert np.max(np.abs(r)) < 1e-6
        assert np.all(np.linalg.norm(G[b][:, ~active], axis=0) <= lam * (1 + 1e-6))


def test_projections():
    K, M = 8, 64
    L = P.mp_edge(K, M)
    assert L == pytest.approx(117.2548, rel=1e-6)
    np.testing.assert_allclose(P.project_eta(np.array([1.0, 0.0, 0.75 / L]), K, M),
                               [1 / L, 1 / (2 * L), 0.75 / L])
    np.testing.assert_array_equal(P.project_lambda(np.array([-1.0, 0.2])), [0.0, 0.2])


def test_paper_pgd_statistics():
    g = _golden("paper_pgd_pcg.txt")
    K, M = int(g["K"]), int(g["M"])
    w = WL.paper_workload(seed=123, B=100, K=K, M=M, gamma_db=g["gamma_db"], sigma=g["sigma"])
    Wzf, _ = O.zf_precoder(w.H, w.gamma_lin, g["sigma"] ** 2, 0.0)
    eta = 1.0 / P.mp_edge(K, M)
    _, hist = P.pgd(w.H, w.gamma_lin, g["sigma"], g["lambda"], eta, 5000, history=True)
    pcg20 = np.mean(P.pcg(Wzf, hist[19]))
    pcg_near = np.mean(P.pcg(Wzf, hist[int(g["pgd_iters_near_optimum"]) - 1]))
    pcg_end = np.mean(P.pcg(Wzf, hist[-1]))
    # 20 iterations: about the consumption of ZF
    assert abs(pcg20 - g["pcg_pgd_20_iter"]) < 0.03
    # after 3500 iterations PGD is close to the optimum's PCG (1.116)
    assert abs(pcg_near - g["pcg_target"]) < 0.02
    assert abs(pcg_end - g["pcg_target"]) < 0.02
    # the unfolded network's 20-layer PCG lies between 20 PGD iterations and the optimum
    assert pcg20 < g["pcg_unfolded_20_layers"] < pcg_end
    # the SINR constraint is (nearly) met: R_sum close to the target 8 log2(11)
    rs = np.mean(P.sum_rate(w.H, hist[-1], g["sigma"] ** 2))
    assert abs(rs - 8 * np.log2(11)) < 0.3
