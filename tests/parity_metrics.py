"""Error measures of a GPU result against the FP64 oracle (test helpers).

rel          normwise ||a - b|| / ||b|| over a whole array (the gate)
rel_per_f    the same per frequency (leading axis), the largest over f
log_err_v    per-bin |ln v_gpu - ln v_oracle|: its 99.9th percentile and
             maximum (v spans orders of magnitude, so a normwise error
             over the array is dominated by the loud bins)
"""
import numpy as np


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def rel_per_f(a, b, axis=0):
    a = np.moveaxis(np.asarray(a), axis, 0)
    b = np.moveaxis(np.asarray(b), axis, 0)
    d = np.linalg.norm((a - b).reshape(a.shape[0], -1), axis=1)
    n = np.linalg.norm(b.reshape(b.shape[0], -1), axis=1)
    return float((d / n).max())


def log_err_v(v, vo):
    e = np.abs(np.log(np.asarray(v, np.float64)) - np.log(np.asarray(vo, np.float64))).ravel()
    return float(np.percentile(e, 99.9)), float(e.max())


def report(g, Po, lo, vo, yo=None):
    """Every measure for one run: g holds the GPU's P, lam, v (and y)."""
    out = dict(v=rel(g["v"], vo), lam=rel(g["lam"], lo), P=rel(g["P"], Po),
               v_f=rel_per_f(g["v"], vo), lam_f=rel_per_f(g["lam"], lo), P_f=rel_per_f(g["P"], Po))
    out["v_log999"], out["v_logmax"] = log_err_v(g["v"], vo)
    if yo is not None and "y" in g:
        out["y"] = max(rel(g["y"][n], yo[n]) for n in range(yo.shape[0]))
        out["y_f"] = max(rel_per_f(g["y"][n], yo[n]) for n in range(yo.shape[0]))
    return out
