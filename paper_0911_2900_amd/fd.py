"""Fundamental diagram from region counts (host post-processing).

The paper picks v_m = 4 because the model then reproduces Weidmann's
fundamental diagram (Sec. 2).  Here the diagram is measured from the counts
that the library records after every step (Context.set_regions): column 0 the
agents in a measurement area of `area_m2`, column 1 the agents upstream of a
line across a corridor of `width_m`.  Agents only move and the upstream end is
closed, so the drop of the upstream count over one step (1 s) is the net flow
across the line.
"""
from __future__ import annotations

import numpy as np


def samples(series: np.ndarray, area_m2: float, width_m: float):
    """(density P/m^2, specific flow P/(m s)) for every step k >= 1 whose rows
    k - 1 and k were recorded; steps with an empty measurement area carry no
    information and are left out."""
    s = np.asarray(series, dtype=np.int64)
    a, u = s[:, 0], s[:, 1]
    ok = (a[1:] >= 0) & (u[1:] >= 0) & (u[:-1] >= 0) & (a[1:] > 0)
    rho = a[1:][ok] / area_m2
    flow = (u[:-1] - u[1:])[ok] / width_m
    return rho, flow


def diagram(rho: np.ndarray, flow: np.ndarray, bin_width: float = 0.25, min_samples: int = 20):
    """Mean and standard deviation of the specific flow per density bin
    [i w, (i + 1) w), for bins with at least min_samples samples."""
    rho, flow = np.asarray(rho, dtype=np.float64), np.asarray(flow, dtype=np.float64)
    out = []
    if len(rho) == 0:
        return out
    idx = np.floor(rho / bin_width).astype(np.int64)
    for b in np.unique(idx):
        m = idx == b
        if m.sum() < min_samples:
            continue
        out.append({"rho_lo": float(b * bin_width), "rho_mean": float(rho[m].mean()),
                    "flow_mean": float(flow[m].mean()), "flow_std": float(flow[m].std()),
                    "samples": int(m.sum())})
    return out


def weidmann_flow(rho: np.ndarray, v0: float = 1.34, gamma: float = 1.913, rho_max: float = 5.4):
    """Specific flow rho * v(rho) of Weidmann's published fit (1993),
    v = v0 (1 - exp(-gamma (1/rho - 1/rho_max))), for context only."""
    rho = np.asarray(rho, dtype=np.float64)
    with np.errstate(divide="ignore"):
        v = v0 * (1.0 - np.exp(-gamma * (1.0 / rho - 1.0 / rho_max)))
    return np.where(rho > 0, rho * np.maximum(v, 0.0), 0.0)
