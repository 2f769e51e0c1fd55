"""Chain analysis of the paper's results section, on host arrays of bead
positions (unwrapped) and centre-of-mass series sampled at LB-step
boundaries.  Plain numpy; no GPU work happens here.

Definitions (Sec. III.A static properties, Sec. III.B dynamic properties):
  * R_g^2 = (1 / 2N^2) sum_ij r_ij^2 and R_e^2 = (r_N - r_1)^2;
  * <1/R_H> = (1/N^2) sum_{i != j} <1/r_ij>;
  * S(k) = (1/N) sum_ij sin(k r_ij) / (k r_ij), and the Flory exponent nu
    from S(k) ~ k^(-1/nu) in the scaling regime;
  * g1(t): mean-square displacement of a monomer (the two innermost), g2(t):
    the same in the centre-of-mass frame, g3(t): of the centre of mass,
    all averaged over time origins t0;
  * D_CM from g3(t) = 6 D_CM t, and tau_tr = <R_g^2> / (6 D_CM);
  * Rouse modes X_p = (1/N) sum_n r_n cos[p pi (n - 1/2) / N], p = 1..N-1,
    and their normalised autocorrelation <X_p(t0 + t) . X_p(t0)> / <X_p^2>.
"""
from __future__ import annotations

import numpy as np


def rg2(x: np.ndarray) -> np.ndarray:
    """Radius of gyration squared in the pair form; x [..., N, 3]."""
    d = x[..., :, None, :] - x[..., None, :, :]
    n = x.shape[-2]
    return np.sum(d * d, axis=(-1, -2, -3)) / (2.0 * n * n)


def inverse_hydrodynamic_radius(x: np.ndarray) -> np.ndarray:
    """<1/R_H> = (1/N^2) sum_{i != j} 1/r_ij (Sec. III.A, the chain's
    hydrodynamic radius in an infinite medium); x [..., N, 3]."""
    n = x.shape[-2]
    d = x[..., :, None, :] - x[..., None, :, :]
    r = np.sqrt(np.sum(d * d, axis=-1))
    off = ~np.eye(n, dtype=bool)
    return np.sum(np.where(off, 1.0 / np.where(off, r, 1.0), 0.0), axis=(-1, -2)) / (n * n)


def re2(x: np.ndarray) -> np.ndarray:
    """End-to-end distance squared; x [..., N, 3]."""
    d = x[..., -1, :] - x[..., 0, :]
    return np.sum(d * d, axis=-1)


def structure_factor(x: np.ndarray, ks: np.ndarray) -> np.ndarray:
    """S(k) for every k in ks, averaged over the leading axes of x [..., N, 3]."""
    n = x.shape[-2]
    d = x[..., :, None, :] - x[..., None, :, :]
    r = np.sqrt(np.sum(d * d, axis=-1)).reshape(-1, n, n)
    out = np.empty(len(ks))
    for i, k in enumerate(ks):
        kr = k * r
        with np.errstate(invalid="ignore", divide="ignore"):
            s = np.where(kr > 0, np.sin(kr) / np.where(kr > 0, kr, 1.0), 1.0)
        out[i] = np.mean(np.sum(s, axis=(-1, -2))) / n
    return out


def power_law_exponent(t: np.ndarray, g: np.ndarray, tmin: float, tmax: float) -> float:
    """Least-squares slope of log g against log t over tmin <= t <= tmax."""
    m = (t >= tmin) & (t <= tmax)
    if np.count_nonzero(m) < 2:
        raise ValueError("fewer than two points in the fit window")
    return float(np.polyfit(np.log(t[m]), np.log(g[m]), 1)[0])


def flory_exponent(ks: np.ndarray, s: np.ndarray, kmin: float, kmax: float) -> float:
    """nu from S(k) ~ k^(-1/nu) over kmin <= k <= kmax."""
    return -1.0 / power_law_exponent(ks, s, kmin, kmax)


def msd(series: np.ndarray, lags: np.ndarray) -> np.ndarray:
    """Mean-square displacement <(y(t0 + lag) - y(t0))^2> over all time
    origins t0 and all leading items; series [T, ..., 3], lags in samples."""
    out = np.empty(len(lags))
    for i, lag in enumerate(lags):
        d = series[lag:] - series[: len(series) - lag]
        out[i] = np.mean(np.sum(d * d, axis=-1))
    return out


def diffusion_constant(t: np.ndarray, g3: np.ndarray, tmin: float, tmax: float) -> float:
    """D from a least-squares fit of g3 = 6 D t (through the origin) over
    tmin <= t <= tmax."""
    m = (t >= tmin) & (t <= tmax)
    if not np.any(m):
        raise ValueError("no points in the fit window")
    return float(np.sum(g3[m] * t[m]) / np.sum(t[m] * t[m]) / 6.0)


def rouse_modes(x: np.ndarray, pmax: int | None = None) -> np.ndarray:
    """X_p for p = 1..pmax (default N-1); x [..., N, 3] -> [..., pmax, 3]."""
    n = x.shape[-2]
    pmax = n - 1 if pmax is None else pmax
    p = np.arange(1, pmax + 1)[:, None]
    c = np.cos(np.pi * p * (np.arange(1, n + 1)[None, :] - 0.5) / n) / n
    return np.einsum("pn,...nc->...pc", c, x)


def autocorrelation(series: np.ndarray, lags: np.ndarray) -> np.ndarray:
    """<y(t0 + lag) . y(t0)> / <y . y> over time origins and leading items;
    series [T, ..., 3]."""
    y0 = np.mean(np.sum(series * series, axis=-1))
    out = np.empty(len(lags))
    for i, lag in enumerate(lags):
        out[i] = np.mean(np.sum(series[lag:] * series[: len(series) - lag], axis=-1)) / y0
    return out


def block_error(samples: np.ndarray, n_blocks: int = 16) -> float:
    """Standard error of the mean of a correlated series [T, ...] from the
    spread of n_blocks contiguous block means (leading axis is time)."""
    t = len(samples) // n_blocks * n_blocks
    if t < n_blocks:
        raise ValueError("series shorter than the number of blocks")
    means = np.mean(samples[:t].reshape(n_blocks, -1), axis=1)
    return float(np.std(means, ddof=1) / np.sqrt(n_blocks))
