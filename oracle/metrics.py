"""Eq. (7): normalised mean absolute error between a result and a reference.

  eps = (1/N) sum_i ||M_i - M~_i|| / Ms

The paper applies it to "the points in the reference dataset"; both readings
are provided: ``epsilon_series`` over a time series of <M> (rows of 3
components) and ``epsilon_map`` over the cells of a magnetization map.
Pins: eps of identical inputs is 0; a uniform offset d gives |d|/Ms.
"""

import numpy as np


def epsilon_series(mavg, mavg_ref, Ms):
    """Eq. (7) over two <M> series sampled at the same times; series of
    different length are an error (the points must correspond)."""
    a = np.asarray(mavg, dtype=np.float64).reshape(-1, 3)
    b = np.asarray(mavg_ref, dtype=np.float64).reshape(-1, 3)
    if len(a) != len(b):
        raise ValueError(f"series of different length: {len(a)} and {len(b)} points")
    return float(np.mean(np.linalg.norm(a - b, axis=1)) / Ms)


def epsilon_map(M, M_ref, Ms):
    d = np.asarray(M, dtype=np.float64) - np.asarray(M_ref, dtype=np.float64)
    return float(np.mean(np.sqrt(np.sum(d * d, axis=0))) / Ms)


def mean_m(M):
    return np.asarray(M, dtype=np.float64).reshape(3, -1).mean(axis=1)
