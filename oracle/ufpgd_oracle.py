"""FP64 oracle of unsupervised training of the unfolded PGD network.

TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline leg of the
benchmark); shares no code with the HIP path.

What is trained (Sec. V, eq. unfoldednet and the unsupervised cost):
  per-layer parameters lambda^(i), eta^(i), i = 0..I-1, of the network
  W^(i+1) = prox_{lambda^(i) eta^(i) ||.||_{2,1}}(W^(i) - eta^(i) grad f(W^(i))),
  W^(0) = H^*, minimising the cost of the output
  C(W^(I)) = lambda_c ||W^(I)||_{2,1} + ||H W^(I)T - sigma D_gamma^{1/2}||_F^2
  with the cost's own lambda_c = 1/15 (Sec. VI-C), averaged over a batch.
Optimiser (Sec. VI-A): Adam (Kingma and Ba, Algorithm 1) with learning rate
1e-3 and batch 64 over 1e5 CN(0, 1) channels; after every update lambda^(i)
is projected onto [0, inf) and eta^(i) into [1/(2 L~), 1/L~] (Sec. V).

Gradients are computed by reverse-mode differentiation of the layer, derived
here by hand.  Conventions: for a real function C of a complex matrix X the
cotangent is Gbar_X = dC/dRe X + j dC/dIm X, so dC = Re sum(conj(Gbar_X) dX).
  cost:       Gbar_W = 2 (H W^T - S)^T H^* + lambda_c w_m / ||w_m||      (S = sigma D^{1/2})
  prox:       w = (1 - t/n) v for n = ||v|| > t, else 0 (identity at t = 0);
              with rho = Re(v^H gbar_w):
              gbar_v = (1 - t/n) gbar_w + (t rho / n^3) v,  dC/dt = -rho / n
  step:       V = W - eta ((W H^T - S) H^*) is complex-linear in W with
              the Hermitian M x M map I - eta H^T H^*, so
              gbar_W = gbar_V - eta (gbar_V H^T) H^*,
              dC/deta = -Re sum(conj(gbar_V) ((W H^T - S) H^*))
  parameters: t = lambda eta, so dC/dlambda = eta dC/dt and dC/deta gains lambda dC/dt.
These are pinned by finite differences and by torch's autograd.

Readings (the paper is silent): the projections act on the stored parameters
after every Adam update; the parameters start at the plain PGD values
lambda^(i) = 1/15 and eta^(i) = 1/L~; early stopping keeps the parameters of
the epoch with the lowest validation cost and stops after `patience` epochs
without improvement; the batch cost is the mean over its channels.
"""
from __future__ import annotations

import numpy as np

from . import pgd_oracle as P


def cost(H, W, gamma, sigma, lam_c):
    """Unsupervised cost per channel (Sec. V): lambda_c ||W||_{2,1} + ||H W^T - S||_F^2."""
    return P.lagrangian(H, W, gamma, sigma, lam_c)


def cost_cotangent(H, W, gamma, sigma, lam_c):
    """Gbar_W of the cost.  A zero column takes the zero subgradient."""
    H = np.asarray(H, np.complex128)
    W = np.asarray(W, np.complex128)
    R = P.residual(H, W, gamma, sigma)                       # [..][K][K]
    G = 2.0 * np.swapaxes(R, -1, -2) @ np.conj(H)
    n = np.sqrt(np.sum(np.abs(W) ** 2, axis=-2, keepdims=True))
    G = G + lam_c * np.where(n > 0, W / np.where(n > 0, n, 1.0), 0.0)
    return G


def forward(H, gamma, sigma, lams, etas, W0=None):
    """The network's forward pass, keeping each layer's input and pre-prox V."""
    H = np.asarray(H, np.complex128)
    W = np.conj(H) if W0 is None else np.asarray(W0, np.complex128)
    tape = []
    for lam, eta in zip(lams, etas):
        V = W - eta * P.wirtinger_gradient(H, W, gamma, sigma)
        tape.append((W, V))
        W = P.prox_l21(V, lam * eta)
    return W, tape


def backward(H, tape, gamma, sigma, lams, etas, gbar):
    """Reverse pass from gbar = Gbar_{W^(I)}: returns dC/dlambda, dC/deta as [..][I]."""
    H = np.asarray(H, np.complex128)
    HT = np.swapaxes(H, -1, -2)
    I = len(tape)
    batch = H.shape[:-2]
    dlam = np.zeros(batch + (I,))
    deta = np.zeros(batch + (I,))
    for i in range(I - 1, -1, -1):
        W, V = tape[i]
        lam, eta = lams[i], etas[i]
        t = lam * eta
        n = np.sqrt(np.sum(np.abs(V) ** 2, axis=-2, keepdims=True))      # [..][1][M]
        rho = np.sum(np.real(np.conj(gbar) * V), axis=-2, keepdims=True)
        active = n > t
        ns = np.where(active, n, 1.0)
        # a column at or below the threshold maps to zero (zero cotangent), except
        # at t = 0, where the prox is the identity
        gv = np.where(active, (1.0 - t / ns) * gbar + (t * rho / ns ** 3) * V,
                      gbar if t == 0 else 0.0)
        dt = -np.sum(np.where(active, rho / ns, 0.0), axis=(-2, -1))
        gf = P.wirtinger_gradient(H, W, gamma, sigma)
        d_eta_step = -np.sum(np.real(np.conj(gv) * gf), axis=(-2, -1))
        gbar = gv - eta * (gv @ HT) @ np.conj(H)
        dlam[..., i] = eta * dt
        deta[..., i] = d_eta_step + lam * dt
    return dlam, deta


def grad(H, gamma, sigma, lams, etas, lam_c, W0=None):
    """Per-channel cost of the network output and its gradients: (C [..], dlam [..][I], deta [..][I])."""
    W, tape = forward(H, gamma, sigma, lams, etas, W0)
    C = cost(H, W, gamma, sigma, lam_c)
    dlam, deta = backward(H, tape, gamma, sigma, lams, etas, cost_cotangent(H, W, gamma, sigma, lam_c))
    return C, dlam, deta


class Adam:
    """Adam (Kingma and Ba 2015, Algorithm 1) on a flat FP64 parameter vector."""

    def __init__(self, n, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0

    def step(self, p, g):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mhat = self.m / (1 - self.b1 ** self.t)
        vhat = self.v / (1 - self.b2 ** self.t)
        return p - self.lr * mhat / (np.sqrt(vhat) + self.eps)


def project(lams, etas, K, M):
    """Parameter projections of Sec. V."""
    return P.project_lambda(lams), P.project_eta(etas, K, M)


def initial_params(I, K, M, lam=1.0 / 15.0):
    """lambda^(i) = 1/15, eta^(i) = 1/L~: the network starts as I iterations of PGD."""
    return np.full(I, lam), np.full(I, 1.0 / P.mp_edge(K, M))


def batch_grad(H, gamma, sigma, lams, etas, lam_c):
    """Mean cost over a batch of channels [B][K][M] and its gradient (dlam [I], deta [I])."""
    C, dl, de = grad(H, gamma, sigma, lams, etas, lam_c)
    return C.mean(), dl.mean(axis=0), de.mean(axis=0)


def train_steps(Htrain, gamma, sigma, lam_c, lams, etas, batches, opt=None, lr=1e-3):
    """Adam steps over the given batches (lists of channel indices into Htrain).

    Returns (lams, etas, opt, batch costs).  Each step: mean gradient over the
    batch, one Adam update of [lambda; eta], then the projections."""
    K, M = Htrain.shape[-2:]
    I = len(lams)
    opt = opt or Adam(2 * I, lr=lr)
    p = np.concatenate([lams, etas]).astype(np.float64)
    costs = []
    for idx in batches:
        C, dl, de = batch_grad(Htrain[idx], gamma, sigma, p[:I], p[I:], lam_c)
        p = opt.step(p, np.concatenate([dl, de]))
        l, e = project(p[:I], p[I:], K, M)
        p = np.concatenate([l, e])
        costs.append(C)
    return p[:I], p[I:], opt, np.asarray(costs)
