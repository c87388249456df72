"""Brute-force (explicit loop) versions of the oracle for tiny inputs.

TEST INFRASTRUCTURE ONLY: they check the vectorised oracle in
dmimo_oracle.py element by element.  Plain Python scalars and loops only, with
``math``/``cmath`` for sqrt and exp, and no numpy arithmetic.  A broadcasting,
transposition or conjugation slip in the vectorised code therefore shows up as
a mismatch.
"""
from __future__ import annotations

import cmath
import math

C = 299_792_458.0


def channel(points, aps, freq_hz, d_min=None):
    lam = C / freq_hz
    if d_min is None or d_min <= 0:
        d_min = lam / (4 * math.pi)
    out = []
    for p in points:
        row = []
        for a in aps:
            d = math.sqrt((p[0] - a[0]) ** 2 + (p[1] - a[1]) ** 2 + (p[2] - a[2]) ** 2)
            amp = lam / (4 * math.pi * max(d, d_min))
            row.append(amp * cmath.exp(-2j * math.pi * d / lam))
        out.append(row)
    return out


def gram(H):
    K = len(H)
    M = len(H[0])
    G = [[0j] * K for _ in range(K)]
    for k in range(K):
        for j in range(K):
            s = 0j
            for m in range(M):
                s += H[k][m] * H[j][m].conjugate()
            G[k][j] = s
    return G


def solve(A, b_cols):
    """Gauss-Jordan elimination with partial pivoting: returns A^{-1} B.

    B is given as a list of rows.
    """
    n = len(A)
    ncol = len(b_cols[0])
    aug = [list(A[i]) + list(b_cols[i]) for i in range(n)]
    for c in range(n):
        piv = max(range(c, n), key=lambda r: abs(aug[r][c]))
        aug[c], aug[piv] = aug[piv], aug[c]
        pv = aug[c][c]
        aug[c] = [v / pv for v in aug[c]]
        for r in range(n):
            if r != c:
                f = aug[r][c]
                aug[r] = [aug[r][i] - f * aug[c][i] for i in range(n + ncol)]
    return [row[n:] for row in aug]


def zf(H, gamma, sigma2, p_total):
    K = len(H)
    M = len(H[0])
    X = solve(gram(H), H)
    if p_total > 0:
        fro2 = sum(abs(X[k][m]) ** 2 for k in range(K) for m in range(M))
        c = [math.sqrt(p_total / fro2)] * K
    else:
        c = [math.sqrt(sigma2) * math.sqrt(gamma[k]) for k in range(K)]
    return [[c[k] * X[k][m].conjugate() for m in range(M)] for k in range(K)]


def mr(H, p_total):
    K = len(H)
    M = len(H[0])
    c = 1.0
    if p_total > 0:
        c = math.sqrt(p_total) / math.sqrt(sum(abs(H[k][m]) ** 2 for k in range(K) for m in range(M)))
    return [[c * H[k][m].conjugate() for m in range(M)] for k in range(K)]


def user_sinr(H, W, sigma2):
    K = len(H)
    M = len(H[0])
    out = []
    for k in range(K):
        sig = 0.0
        intf = 0.0
        for j in range(K):
            a = sum(H[k][m] * W[j][m] for m in range(M))
            if j == k:
                sig = abs(a) ** 2
            else:
                intf += abs(a) ** 2
        out.append(sig / (intf + sigma2))
    return out


def maps(Hpts, W, sigma2):
    """Returns (power, sinr, best_k, per_stream) lists for every point."""
    K = len(W)
    M = len(W[0])
    power, sinr, best, per = [], [], [], []
    for row in Hpts:
        z = [sum(row[m] * W[k][m] for m in range(M)) for k in range(K)]
        p = [abs(v) ** 2 for v in z]
        y = sum(p)
        bk = 0
        bs = -1.0
        for k in range(K):
            s = p[k] / (sum(p[j] for j in range(K) if j != k) + sigma2)
            if s > bs:
                bs = s
                bk = k
        power.append(y)
        sinr.append(bs)
        best.append(bk)
        per.append(p)
    return power, sinr, best, per


def antenna_power(W):
    K = len(W)
    M = len(W[0])
    return [sum(abs(W[k][m]) ** 2 for k in range(K)) for m in range(M)]
