"""FP64 oracle of the PA-consumption-aware precoder on an arbitrary deployment.

TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline leg of the
benchmark); shares no code with the HIP path.

The paper solves eq. (optim1) (Sec. III) with PGD / unfolded PGD (Sec. IV-V)
for unit-variance Rayleigh channels and unit noise, and sets the step from
the Marchenko-Pastur edge of such channels.  A distributed deployment has
channels of any scale and correlation.  Reading used here (the paper is
silent on other channels):
  1. normalise: s = RMS |h_km|, Hn = H / s, unit noise (sigma_n = 1), so
     lambda keeps the meaning it has in the paper (1/15);
  2. step: eta_i = eta_rel_i / L with L = the largest eigenvalue of Hn Hn^H
     (= that of Hn^T Hn^*, the Lipschitz constant of Sec. IV), computed per
     deployment instead of the Marchenko-Pastur approximation;
  3. solve with W(0) = Hn^*, then map back: W = (sigma / s) Wn.
Step 3 is exact for the constraint: H W^T = sigma Hn Wn^T, so a solution of
Hn Wn^T = D^{1/2} gives H W^T = sigma D^{1/2} (eq. optim1).
"""
from __future__ import annotations

import numpy as np

from . import dmimo_oracle as O
from . import pgd_oracle as P


def normalisation(H):
    """s = RMS |h_km| and L = lambda_max(Hn Hn^H) per deployment ([..][K][M])."""
    H = np.asarray(H, np.complex128)
    s = np.sqrt(np.mean(np.abs(H) ** 2, axis=(-2, -1)))
    Hn = H / s[..., None, None]
    G = Hn @ np.conj(np.swapaxes(Hn, -1, -2))
    L = np.linalg.eigvalsh(G)[..., -1]
    return s, L


def pa_precoder(H, gamma, sigma2, lams, eta_rel):
    """W [..][K][M] of the PA-aware precoder (layers lams, eta_rel) in the
    deployment's own units; also returns (s, L)."""
    H = np.asarray(H, np.complex128)
    s, L = normalisation(H)
    Hn = H / s[..., None, None]
    batch = H.shape[:-2]
    Wn = np.empty_like(Hn)
    for b in np.ndindex(*batch) if batch else [()]:
        etas = np.asarray(eta_rel, np.float64) / L[b]
        Wn[b] = P.unfolded(Hn[b], gamma, 1.0, lams, etas)
    sig = np.sqrt(sigma2)
    return (sig / s)[..., None, None] * Wn, s, L
