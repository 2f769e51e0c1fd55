"""Chain analysis functions against closed forms (no GPU)."""
from __future__ import annotations

import numpy as np
import pytest

from paper_0903_5067_amd import analysis as an


def _straight(n, a=1.0):
    x = np.zeros((n, 3))
    x[:, 0] = a * np.arange(n)
    return x


def test_rg2_re2_of_a_straight_chain():
    """Rod of N beads spaced a: R_g^2 = a^2 (N^2 - 1) / 12, R_e^2 = a^2 (N - 1)^2."""
    for n in (2, 7, 32):
        x = _straight(n, 0.97)
        assert an.rg2(x) == pytest.approx(0.97 ** 2 * (n * n - 1) / 12, rel=1e-13)
        assert an.re2(x) == pytest.approx(0.97 ** 2 * (n - 1) ** 2, rel=1e-13)


def test_inverse_hydrodynamic_radius_of_a_rod():
    """Rod of N beads spaced a: (1/N^2) sum_{i != j} 1/(a |i - j|)
    = 2 (N H_{N-1} - (N - 1)) / (a N^2), H the harmonic number."""
    for n in (2, 7, 32):
        x = _straight(n, 0.97)
        h = sum(1.0 / m for m in range(1, n))
        assert an.inverse_hydrodynamic_radius(x) == pytest.approx(2 * (n * h - (n - 1)) / (0.97 * n * n), rel=1e-13)


def test_rg2_pair_form_equals_centre_of_mass_form():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(5, 32, 3))
    com = x.mean(axis=1, keepdims=True)
    ref = np.mean(np.sum((x - com) ** 2, axis=-1), axis=1)
    np.testing.assert_allclose(an.rg2(x), ref, rtol=1e-12)


def test_structure_factor_limits_and_dimer():
    """S(0) = N; a dimer at distance d: S = 1 + sin(kd)/(kd)."""
    x = np.array([[0.0, 0, 0], [1.3, 0, 0]])
    ks = np.array([1e-9, 0.7, 2.5])
    s = an.structure_factor(x, ks)
    assert s[0] == pytest.approx(2.0, rel=1e-12)
    for k, v in zip(ks[1:], s[1:]):
        assert v == pytest.approx(1 + np.sin(k * 1.3) / (k * 1.3), rel=1e-12)


def test_power_law_and_flory_fits_on_exact_power_laws():
    t = np.geomspace(1, 1000, 40)
    assert an.power_law_exponent(t, 3.0 * t ** 0.675, 20, 80) == pytest.approx(0.675, rel=1e-12)
    ks = np.geomspace(0.5, 5, 20)
    assert an.flory_exponent(ks, 7.0 * ks ** (-1 / 0.617), 1, 3) == pytest.approx(0.617, rel=1e-12)


def test_msd_of_uniform_motion_and_diffusion_fit():
    """y(t) = v t: MSD(lag) = |v|^2 lag^2; g3 = 6 D t is recovered exactly."""
    v = np.array([0.3, -0.2, 0.1])
    y = np.arange(50)[:, None] * v
    lags = np.array([1, 3, 10])
    np.testing.assert_allclose(an.msd(y, lags), np.sum(v * v) * lags ** 2, rtol=1e-12)
    t = np.linspace(1, 100, 50)
    assert an.diffusion_constant(t, 6 * 5.162e-3 * t, 20, 80) == pytest.approx(5.162e-3, rel=1e-12)


def test_rouse_modes_orthogonality():
    """A chain shaped as the q-th cosine projects on X_q = e_x / 2 only."""
    n, q = 32, 3
    x = np.zeros((n, 3))
    x[:, 0] = np.cos(np.pi * q * (np.arange(1, n + 1) - 0.5) / n)
    xp = an.rouse_modes(x)
    expect = np.zeros((n - 1, 3))
    expect[q - 1, 0] = 0.5
    np.testing.assert_allclose(xp, expect, atol=1e-14)


def test_autocorrelation_of_an_exponential_sequence():
    """y(t) = e^{-t/tau} e_x: the estimator equals its definition written out
    on the finite series, and is 1 at lag 0."""
    tau = 5.0
    t = np.arange(400)
    y = np.zeros((400, 3))
    y[:, 0] = np.exp(-t / tau)
    lags = np.array([0, 2, 7])
    got = an.autocorrelation(y, lags)
    ref = [np.mean(y[l:, 0] * y[: 400 - l, 0]) / np.mean(y[:, 0] ** 2) for l in lags]
    np.testing.assert_allclose(got, ref, rtol=1e-12)
    assert got[0] == 1.0


def test_block_error():
    assert an.block_error(np.full((64, 3), 2.5)) == 0.0
    rng = np.random.default_rng(7)
    s = rng.normal(size=(20000, 4))
    # independent samples: close to sigma / sqrt(n)
    assert an.block_error(s) == pytest.approx(1 / np.sqrt(s.size), rel=0.5)


def test_rouse_analysis_recovers_rouse_chain_relaxation_times():
    """Sec. III.B validates its Rouse-mode analysis on a Gaussian Rouse chain
    of N = 8 without hydrodynamics or excluded volume.  Here: 400 such chains
    (harmonic springs k, friction zeta, overdamped Langevin, Euler-Maruyama).
    The X_p of the paper's definition are the exact normal modes of this
    chain, with <X_p(t) . X_p(0)> / <X_p^2> = exp(-t / tau_p) and
    tau_p = zeta / (4 k sin^2(p pi / 2N)).  The analysis functions give tau_p
    to the statistical error."""
    rng = np.random.default_rng(11)
    n_ch, N, k, zeta, kT, dt = 400, 8, 1.0, 1.0, 1.0, 0.005
    every, n_samp = 10, 2000
    x = np.cumsum(rng.normal(scale=np.sqrt(kT / k), size=(n_ch, N, 3)), axis=1)   # equilibrium bonds
    amp = np.sqrt(2 * kT * dt / zeta)
    series = np.empty((n_samp, n_ch, N, 3))
    for i in range(n_samp):
        for _ in range(every):
            f = np.zeros_like(x)
            bond = x[:, 1:] - x[:, :-1]
            f[:, :-1] += k * bond
            f[:, 1:] -= k * bond
            x = x + f * (dt / zeta) + amp * rng.normal(size=x.shape)
        series[i] = x
    modes = an.rouse_modes(series, 5)                       # [T, chains, 5, 3]
    t_s = every * dt
    for p in range(1, 6):
        tau = zeta / (4 * k * np.sin(p * np.pi / (2 * N)) ** 2)
        lags = np.arange(0, int(tau / t_s) + 1)             # the ACF from 1 down to ~1/e
        c = an.autocorrelation(modes[:, :, p - 1], lags)
        slope = np.polyfit(lags * t_s, np.log(c), 1)[0]
        assert -1.0 / slope == pytest.approx(tau, rel=0.03), p
