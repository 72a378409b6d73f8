"""Comparison helpers for (value, exponent) series of the library and the oracle."""
from __future__ import annotations

import numpy as np


def rel_err_series(g_val, g_exp, o_val, o_exp, floor=1e-30):
    """Max relative error of g_val*2^g_exp against o_val*2^o_exp over entries whose
    magnitude exceeds floor * the largest magnitude (log-safe: no underflow)."""
    g_val = np.asarray(g_val, dtype=np.float64)
    o_val = np.asarray(o_val, dtype=np.float64)
    g_exp = np.broadcast_to(np.asarray(g_exp), g_val.shape)
    o_exp = np.broadcast_to(np.asarray(o_exp), o_val.shape)
    gv = np.ldexp(g_val, (g_exp - o_exp).astype(np.int64))        # in the oracle's scale
    # magnitude of every oracle entry as log2
    with np.errstate(divide="ignore"):
        lg = np.where(o_val != 0, np.log2(np.abs(o_val)) + o_exp, -np.inf)
    top = lg.max() if lg.size else -np.inf
    keep = lg > top + np.log2(floor)
    if not keep.any():
        return 0.0
    err = np.abs(gv[keep] - o_val[keep]) / np.abs(o_val[keep])
    return float(err.max())


def rel_l1(g, g_exp, o, o_exp):
    """Relative L1 error of a state g*2^g_exp against o*2^o_exp."""
    g = np.asarray(g, dtype=np.float64)
    o = np.asarray(o, dtype=np.float64)
    gv = np.ldexp(g, int(g_exp) - int(o_exp))
    den = np.abs(o).sum()
    return float(np.abs(gv - o).sum() / den) if den > 0 else float(np.abs(gv).sum())


def oracle_series(r):
    """Oracle run dict -> (tot, tot_exp, det, det_exp) as arrays [T, 3] / [T, n_det]."""
    return r["tot"], r["tot_exp"], r["det"], r["det_exp"]
