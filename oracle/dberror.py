"""Error report in dB against the FP64 oracle.

TEST INFRASTRUCTURE ONLY (the tests and the CPU baseline leg of the
benchmark).

A relative criterion has no bound where the oracle value goes to zero, at ZF
nulls and interference minima.  So a tolerance of ``tol_db`` applies down to
``floor_rel`` (default 1e-6, i.e. -60 dB) below the largest oracle value, and
an absolute floor applies below that:

    |y - y_ref| <= (10^(tol_db/10) - 1) * max(y_ref, floor_rel * max(y_ref))

Per-user SINR values use the plain dB error (floor_rel = 0).
"""
from __future__ import annotations

import numpy as np


def db_error(y, y_ref, floor_rel: float = 1e-6):
    """Per-element |10 log10(y / y_ref)| for points above the floor.

    Points below the floor get NaN.  Returns (err_db [N], above_floor mask).
    """
    y = np.asarray(y, np.float64).ravel()
    r = np.asarray(y_ref, np.float64).ravel()
    floor = floor_rel * np.max(np.abs(r)) if r.size else 0.0
    above = r > floor
    err = np.full(r.shape, np.nan)
    with np.errstate(divide="ignore", invalid="ignore"):
        err[above] = np.abs(10.0 * np.log10(y[above] / r[above]))
    return err, above


def within_db(y, y_ref, tol_db: float, floor_rel: float = 1e-6):
    """Element-wise pass/fail of the floor rule (True = within tolerance)."""
    y = np.asarray(y, np.float64).ravel()
    r = np.asarray(y_ref, np.float64).ravel()
    floor = floor_rel * np.max(np.abs(r)) if r.size else 0.0
    lim = (10.0 ** (tol_db / 10.0) - 1.0) * np.maximum(r, floor)
    return np.abs(y - r) <= lim


def summary(y, y_ref, tol_db: float, floor_rel: float = 1e-6) -> dict:
    """Max and p99 dB error above the floor, the number of points below it,
    and the number of points that break the floor rule."""
    err, above = db_error(y, y_ref, floor_rel)
    ok = within_db(y, y_ref, tol_db, floor_rel)
    e = err[above]
    return {
        "max_db": float(np.max(e)) if e.size else 0.0,
        "p99_db": float(np.percentile(e, 99)) if e.size else 0.0,
        "n": int(err.size),
        "n_below_floor": int(np.count_nonzero(~above)),
        "n_fail": int(np.count_nonzero(~ok)),
        "tol_db": tol_db,
    }
