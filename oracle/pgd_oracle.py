"""FP64 oracle of the paper's solver: proximal gradient descent (PGD) for the
PA-consumption-aware ZF problem, and its deep-unfolded form.

TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline leg of the
benchmark); shares no code with the HIP path.

Problem (Sec. III, eq. optim1 and eq. l): minimise the PA consumed power
alpha ||W||_{2,1} subject to H W^T = sigma D_gamma^{1/2}.  The Lagrangian is
lambda ||W||_{2,1} + ||H W^T - sigma D_gamma^{1/2}||_F^2 (up to the factor mu).

PGD (Sec. IV, eq. proxgd), with the steps in the paper's order:
  1. gradient step with the complex (Wirtinger) gradient
     df/dW^* = W H^T H^* - sigma D_gamma^{1/2} H^*:
        V = W - eta (W H^T H^* - sigma D_gamma^{1/2} H^*);
  2. the proximal operator of lambda eta ||.||_{2,1} applied to the stacked
     real matrix [V_Re; V_Im], column by column:
        w_m = (1 - lambda eta / max(||v_m||_2, lambda eta)) v_m.
     The norm of a stacked column equals the complex column norm, so the
     prox acts on the complex columns directly.
The unfolded network (Sec. V, eq. unfoldednet) is the same iteration with a
per-layer lambda^(i), eta^(i).  eta is projected into [1/(2 L~), 1/L~] with
the Marchenko-Pastur edge L~ = (sqrt K + sqrt M)^2 (Sec. V).

Reading (the paper is silent): sigma is the noise standard deviation,
sqrt(sigma2).  Because the step uses the Wirtinger gradient, which is half
the real gradient of f, a fixed point of the iteration satisfies the
optimality conditions of f/2 + lambda ||W||_{2,1}:
  for a nonzero column: (df/dW^*)_m + lambda w_m / ||w_m|| = 0;
  for a zero column: ||(df/dW^*)_m|| <= lambda.
The tests check exactly this.

Metrics (Sec. VI-B): sum rate R_sum and the power consumption gain
PCG = p_cons^ZF / p_cons = ||W_ZF||_{2,1} / ||W||_{2,1} (alpha cancels).
"""
from __future__ import annotations

import numpy as np

from . import dmimo_oracle as O


def mp_edge(K: int, M: int) -> float:
    """Marchenko-Pastur upper edge L~ = (sqrt K + sqrt M)^2 (Sec. V)."""
    return (np.sqrt(K) + np.sqrt(M)) ** 2


def project_eta(eta, K: int, M: int):
    """eta projected into [1/(2 L~), 1/L~] (Sec. V)."""
    L = mp_edge(K, M)
    return np.minimum(np.maximum(eta, 1.0 / (2.0 * L)), 1.0 / L)


def project_lambda(lam):
    """lambda projected onto [0, inf) (Sec. V)."""
    return np.maximum(lam, 0.0)


def residual(H, W, gamma, sigma):
    """H W^T - sigma D_gamma^{1/2}.  [..][K][K]."""
    H = np.asarray(H, np.complex128)
    K = H.shape[-2]
    target = sigma * np.diag(np.sqrt(np.asarray(gamma, np.float64) * np.ones(K)))
    return O.user_gains(H, W) - target


def smooth_term(H, W, gamma, sigma):
    """f(W) = ||H W^T - sigma D_gamma^{1/2}||_F^2."""
    R = residual(H, W, gamma, sigma)
    return np.sum(np.abs(R) ** 2, axis=(-2, -1))


def lagrangian(H, W, gamma, sigma, lam):
    """lambda ||W||_{2,1} + ||H W^T - sigma D_gamma^{1/2}||_F^2 (eq. l / unsupervised loss)."""
    return lam * O.l21_norm(W) + smooth_term(H, W, gamma, sigma)


def wirtinger_gradient(H, W, gamma, sigma):
    """df/dW^* = W H^T H^* - sigma D_gamma^{1/2} H^* (Sec. IV)."""
    H = np.asarray(H, np.complex128)
    W = np.asarray(W, np.complex128)
    K = H.shape[-2]
    d = sigma * np.sqrt(np.asarray(gamma, np.float64) * np.ones(K))
    HT = np.swapaxes(H, -1, -2)
    return W @ HT @ np.conj(H) - d[:, None] * np.conj(H)


def prox_l21(V, t):
    """Column-wise group soft threshold: (1 - t / max(||v_m||, t)) v_m.

    With t = 0 the operator is the identity (the formula's 0/0 on a zero
    column reads as no shrinkage)."""
    V = np.asarray(V, np.complex128)
    if t == 0:
        return V
    norms = np.sqrt(np.sum(np.abs(V) ** 2, axis=-2, keepdims=True))
    return (1.0 - t / np.maximum(norms, t)) * V


def pgd_layer(H, W, gamma, sigma, lam, eta):
    """One iteration / layer (eq. proxgd, eq. unfoldednet)."""
    V = W - eta * wirtinger_gradient(H, W, gamma, sigma)
    return prox_l21(V, lam * eta)


def unfolded(H, gamma, sigma, lams, etas, W0=None, history=False):
    """Layers i = 0..I-1 with lambda^(i), eta^(i), starting from W^(0) = H^* (Sec. VI-C)."""
    H = np.asarray(H, np.complex128)
    W = np.conj(H) if W0 is None else np.asarray(W0, np.complex128)
    hist = []
    for lam, eta in zip(lams, etas):
        W = pgd_layer(H, W, gamma, sigma, lam, eta)
        if history:
            hist.append(W)
    return (W, hist) if history else W


def pgd(H, gamma, sigma, lam, eta, iters, W0=None, history=False):
    """Plain PGD: the same layer with a fixed lambda and eta."""
    return unfolded(H, gamma, sigma, [lam] * iters, [eta] * iters, W0, history)


def pcg(W_zf, W):
    """PCG = ||W_ZF||_{2,1} / ||W||_{2,1} (Sec. VI-B)."""
    return O.l21_norm(W_zf) / O.l21_norm(W)


def sum_rate(H, W, sigma2):
    return O.sum_rate(O.user_sinr(H, W, sigma2))
