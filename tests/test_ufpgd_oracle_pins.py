"""Pins of the FP64 training oracle (unfolded PGD, Sec. V; training, Sec. VI-A).

The reverse pass is derived by hand in the oracle.  It is pinned to central
finite differences of the oracle's own forward pass, including columns that
the prox sets to zero, and to torch's autograd through a separately written
torch forward pass.  The optimiser is pinned to torch.optim.Adam.
"""
import numpy as np
import pytest

from oracle import pgd_oracle as P
from oracle import ufpgd_oracle as U


def _cn(rng, shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2)


def _tiny_case():
    """K=3, M=5, I=4 with thresholds large enough that some columns are zeroed."""
    rng = np.random.default_rng(11)
    H = _cn(rng, (3, 5))
    gamma = np.array([2.0, 4.0, 3.0])
    sigma = 0.8
    lams = np.array([27.5, 4.3, 2.7, 2.6])
    etas = np.array([0.05, 0.07, 0.06, 0.04])
    return H, gamma, sigma, lams, etas, 0.3


def _fd(f, x, h=1e-6):
    out = np.zeros_like(x)
    for i in range(x.size):
        e = np.zeros_like(x)
        e.flat[i] = h
        out.flat[i] = (f(x + e) - f(x - e)) / (2 * h)
    return out


def test_tiny_case_has_active_and_zeroed_columns_away_from_kinks():
    H, gamma, sigma, lams, etas, lam_c = _tiny_case()
    _, tape = U.forward(H, gamma, sigma, lams, etas)
    zeroed = active = 0
    for (W, V), lam, eta in zip(tape, lams, etas):
        n = np.linalg.norm(V, axis=0)
        t = lam * eta
        assert np.min(np.abs(n - t)) > 1e-3          # no column at the kink of the prox
        zeroed += np.sum(n < t)
        active += np.sum(n > t)
    assert zeroed >= 3 and active >= 3


def test_parameter_gradients_match_finite_differences():
    H, gamma, sigma, lams, etas, lam_c = _tiny_case()
    C, dl, de = U.grad(H, gamma, sigma, lams, etas, lam_c)

    def cost_of(l, e):
        W, _ = U.forward(H, gamma, sigma, l, e)
        return U.cost(H, W, gamma, sigma, lam_c)

    fd_l = _fd(lambda l: cost_of(l, etas), lams)
    fd_e = _fd(lambda e: cost_of(lams, e), etas)
    np.testing.assert_allclose(dl, fd_l, rtol=1e-6, atol=1e-9)
    np.testing.assert_allclose(de, fd_e, rtol=1e-6, atol=1e-9)
    assert np.all(np.abs(de) > 1e-3) and np.all(np.abs(dl) > 1e-3)    # not vacuous


def test_batch_gradient_is_the_gradient_of_the_batch_mean_cost():
    rng = np.random.default_rng(18)
    H = _cn(rng, (4, 3, 7))
    gamma, sigma, lam_c = np.array([2.0, 1.0, 3.0]), 1.1, 0.25
    lams = np.array([0.5, 1.5, 0.2])
    etas = np.array([0.04, 0.05, 0.03])
    C, dl, de = U.batch_grad(H, gamma, sigma, lams, etas, lam_c)

    def mean_cost(l, e):
        W, _ = U.forward(H, gamma, sigma, l, e)
        return U.cost(H, W, gamma, sigma, lam_c).mean()

    assert abs(C - mean_cost(lams, etas)) < 1e-12
    np.testing.assert_allclose(dl, _fd(lambda l: mean_cost(l, etas), lams), rtol=1e-6, atol=1e-9)
    np.testing.assert_allclose(de, _fd(lambda e: mean_cost(lams, e), etas), rtol=1e-6, atol=1e-9)


def test_initial_network_is_twenty_pgd_iterations_at_pcg_one():
    """The network starts as plain PGD (lambda = 1/15, eta = 1/L~), which after
    20 iterations consumes about as much PA power as ZF: PCG close to 1 (Sec. VI-C)."""
    from oracle import dmimo_oracle as O
    rng = np.random.default_rng(17)
    K, M = 8, 64
    H = _cn(rng, (1000, K, M))
    lams, etas = U.initial_params(20, K, M)
    W, _ = U.forward(H, 10.0, 1.0, lams, etas)
    Wzf, _ = O.zf_precoder(H, np.full(K, 10.0), 1.0, 0.0)
    assert abs(P.pcg(Wzf, W).mean() - 1.0) < 0.02
    np.testing.assert_allclose(lams, 1.0 / 15.0)


def test_zero_threshold_layer_is_the_plain_gradient_step():
    """lambda^(i) = 0 (the projection's lower bound) makes the prox the identity,
    also on a column that is exactly zero; its reverse pass is then that of the
    linear gradient step alone."""
    rng = np.random.default_rng(19)
    H = _cn(rng, (2, 4))
    H[:, 1] = 0.0                                    # column 1 of V stays exactly zero
    W0 = _cn(rng, (2, 4))
    W0[:, 1] = 0.0
    gamma, sigma = np.array([1.0, 2.0]), 1.0
    W, tape = U.forward(H, gamma, sigma, [0.0], [0.05], W0=W0)
    np.testing.assert_array_equal(W, tape[0][1])
    assert np.all(np.isfinite(W)) and np.all(W[:, 1] == 0)
    gbar = _cn(rng, (2, 4))
    dl, de = U.backward(H, tape, gamma, sigma, [0.0], [0.05], gbar)
    gf = P.wirtinger_gradient(H, W0, gamma, sigma)
    assert abs(de[0] + np.sum(np.real(np.conj(gbar) * gf))) < 1e-12
    rho = np.sum(np.real(np.conj(gbar) * W), axis=0)
    n = np.linalg.norm(W, axis=0)
    keep = n > 0
    assert abs(dl[0] - 0.05 * -np.sum(rho[keep] / n[keep])) < 1e-12


def test_cost_cotangent_matches_finite_differences():
    rng = np.random.default_rng(12)
    H = _cn(rng, (3, 6))
    W = _cn(rng, (3, 6))
    W[:, 2] = 0.0                                    # a zero column takes the zero subgradient
    gamma, sigma, lam_c = np.array([1.0, 2.0, 5.0]), 0.9, 0.4
    G = U.cost_cotangent(H, W, gamma, sigma, lam_c)
    keep = [m for m in range(6) if m != 2]
    f = lambda x: U.cost(H, x, gamma, sigma, lam_c)
    for k in range(3):
        for m in keep:
            e = np.zeros_like(W)
            e[k, m] = 1e-6
            dre = (f(W + e) - f(W - e)) / 2e-6
            dim = (f(W + 1j * e) - f(W - 1j * e)) / 2e-6
            assert abs(G[k, m].real - dre) < 1e-6 and abs(G[k, m].imag - dim) < 1e-6
    assert np.all(G[:, 2] == 2.0 * (P.residual(H, W, gamma, sigma).T @ np.conj(H))[:, 2])


def test_parameter_gradients_match_torch_autograd_at_paper_size():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(13)
    B, K, M, I = 3, 8, 64, 20
    H = _cn(rng, (B, K, M))
    gamma, sigma, lam_c = np.full(K, 10.0), 1.0, 1.0 / 15.0
    lams = rng.uniform(0.0, 0.6, I)
    etas = P.project_eta(rng.uniform(0.4, 1.1, I) / P.mp_edge(K, M), K, M)
    C, dl, de = U.grad(H, gamma, sigma, lams, etas, lam_c)

    Ht = torch.from_numpy(H)
    lt = torch.tensor(lams, requires_grad=True)
    et = torch.tensor(etas, requires_grad=True)
    d = torch.from_numpy(sigma * np.sqrt(gamma)).to(torch.complex128)
    W = Ht.conj()
    for i in range(I):
        grad_f = (W @ Ht.transpose(-1, -2) - torch.diag(d)) @ Ht.conj()
        V = W - et[i] * grad_f
        n = torch.sqrt((V.real ** 2 + V.imag ** 2).sum(dim=-2, keepdim=True))
        thr = lt[i] * et[i]
        W = (1 - thr / torch.maximum(n, thr)) * V
    R = W @ Ht.transpose(-1, -2) - torch.diag(d)
    cost = lam_c * torch.sqrt((W.real ** 2 + W.imag ** 2).sum(dim=-2)).sum(dim=-1) \
        + (R.real ** 2 + R.imag ** 2).sum(dim=(-2, -1))
    cost.sum().backward()
    np.testing.assert_allclose(C, cost.detach().numpy(), rtol=1e-12)
    np.testing.assert_allclose(dl.sum(axis=0), lt.grad.numpy(), rtol=1e-8, atol=1e-12)
    np.testing.assert_allclose(de.sum(axis=0), et.grad.numpy(), rtol=1e-8, atol=1e-12)


def test_adam_matches_torch_optimiser():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(14)
    p0 = rng.standard_normal(40)
    grads = rng.standard_normal((30, 40)) * np.logspace(-4, 1, 40)
    opt = U.Adam(40, lr=1e-3)
    p = p0.copy()
    tp = torch.tensor(p0, requires_grad=True)
    topt = torch.optim.Adam([tp], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    for g in grads:
        p = opt.step(p, g)
        tp.grad = torch.from_numpy(g.copy())
        topt.step()
    np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-12, atol=1e-15)


def test_projections_hold_after_every_step():
    rng = np.random.default_rng(15)
    K, M, I = 8, 64, 20
    H = _cn(rng, (256, K, M))
    lams, etas = U.initial_params(I, K, M)
    batches = [rng.permutation(256)[:64] for _ in range(5)]
    l, e, opt, costs = U.train_steps(H, 10.0, 1.0, 1.0 / 15.0, lams, etas, batches, lr=0.05)
    L = P.mp_edge(K, M)
    assert np.all(l >= 0.0)
    assert np.all(e >= 1.0 / (2 * L) - 1e-18) and np.all(e <= 1.0 / L + 1e-18)
    assert opt.t == 5 and len(costs) == 5


def test_training_lowers_the_held_out_cost():
    """A few hundred Adam steps from the PGD start lower the unsupervised cost of
    the 20-layer network on channels it was not trained on."""
    rng = np.random.default_rng(16)
    K, M, I = 8, 64, 20
    Htr = _cn(rng, (2048, K, M))
    Hte = _cn(rng, (256, K, M))
    lams, etas = U.initial_params(I, K, M)

    def held_out(l, e):
        W, _ = U.forward(Hte, 10.0, 1.0, l, e)
        return U.cost(Hte, W, 10.0, 1.0, 1.0 / 15.0).mean()

    before = held_out(lams, etas)
    batches = [rng.permutation(2048)[:64] for _ in range(150)]
    l, e, _, _ = U.train_steps(Htr, 10.0, 1.0, 1.0 / 15.0, lams, etas, batches, lr=1e-2)
    after = held_out(l, e)
    assert after < before * 0.99
