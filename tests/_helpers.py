"""Shared test helpers: workload <-> device tensors, error norms."""
from __future__ import annotations

import numpy as np


def rel_inf(x, ref) -> float:
    """max |x - ref| / max |ref| over the whole stacked output."""
    x = np.asarray(x, np.float64).reshape(-1)
    ref = np.asarray(ref, np.float64).reshape(-1)
    den = np.abs(ref).max()
    return float(np.abs(x - ref).max() / (den if den > 0 else 1.0))


def structure(wl):
    """Host structure arrays of a workload: sys_body_ptr, body_trg_ptr, body_src_ptr."""
    n_trg = [wl.shapes[s].trg.shape[0] for s in wl.shape_of_body]
    n_src = [wl.shapes[s].src.shape[0] for s in wl.shape_of_body]
    return (np.asarray(wl.sys_body_ptr, np.int64), np.concatenate([[0], np.cumsum(n_trg)]).astype(np.int64),
            np.concatenate([[0], np.cumsum(n_src)]).astype(np.int64))


def net_flat(wl):
    return np.concatenate([np.asarray(n, np.float64).reshape(-1) for n in wl.net])
