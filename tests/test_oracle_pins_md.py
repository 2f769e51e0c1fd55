"""Pins of the oracle's MD substep and of its negative-population count.

The paper fixes the MD step (Sec. II.E, time steps) but not the integrator;
the reading is velocity Verlet inside each LB step.  Without friction and
noise (zeta = 0, kT = 0) a bead-spring chain is a conservative Hamiltonian
system under the potentials of Sec. II.A, and velocity Verlet then has two
properties a wrong step order lacks: the total energy shows no drift, and its
fluctuation is second order, shrinking four-fold when the step is halved.
Planted copies of the oracle with the substep reordered (conservative force
before the drift) or reduced to first order (a single kick after the drift)
are built on the CPU and must fail the same check.

Sec. II.E (choice of parameters) picks the LB step so that populations n_i
rarely go negative; the oracle counts them (reading: never clipped).  The
count is pinned on hand-made states whose count is known by construction.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np
import pytest

import lbinputs

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE_SRC = os.path.join(os.path.dirname(HERE), "oracle", "lbmd_oracle.cpp")


def _potential(p, x):
    """FENE along the chain plus LJ cut and shifted at 2^(1/6) sigma between
    all pairs, minimum image (Sec. II.A), vectorised."""
    L = p["L"]
    d = x[1:] - x[:-1]
    r2 = np.einsum("ij,ij->i", d, d)
    u = np.sum(-0.5 * p["k_fene"] * p["r0_fene"] ** 2 * np.log(1.0 - r2 / p["r0_fene"] ** 2))
    D = x[:, None, :] - x[None, :, :]
    D -= L * np.round(D / L)
    iu = np.triu_indices(len(x), 1)
    R2 = np.einsum("ijk,ijk->ij", D, D)[iu]
    m = R2 <= 2 ** (1 / 3) * p["sigma_wca"] ** 2
    s6 = (p["sigma_wca"] ** 2 / R2[m]) ** 3
    return u + np.sum(4.0 * p["eps_wca"] * (s6 * s6 - s6 + 0.25))


def _energy_series(run_one, p, x0, v0, n_lb):
    """Total energy at every LB-step boundary of a free chain."""
    st = run_one(p, x0, v0)
    E = []
    for _ in range(n_lb + 1):
        x, v = st.x, st.v
        E.append(0.5 * p["mass"] * float(np.sum(v * v)) + _potential(p, x))
        st.run(1)
    return np.array(E)


SEEDS = (1, 2, 3, 4)


def _verlet_check(run_one, seeds=SEEDS, n_lb=1000):
    """Per seed, (fluctuation, drift, largest excursion) of the total energy of
    a free 16-bead chain over 10^4 MD steps of dt = 0.01 (1000 LB steps of 10
    substeps) and over the same physical time at dt/2 (20 substeps), with the
    initial kinetic energy.  Several seeds: the dt and dt/2 trajectories part
    ways chaotically, so one seed's fluctuation ratio scatters by ~20 %."""
    L, N = 8, 16
    out = []
    for seed in seeds:
        x0 = lbinputs.saw_chain(N, L, seed)
        v0 = np.random.default_rng(seed).normal(size=x0.shape)
        v0 -= v0.mean(axis=0)
        per = []
        for dt, sub in ((0.01, 10), (0.005, 20)):
            p = lbinputs.box_params("plain16", L=L, N=N, kT=0.0, zeta=0.0, md_dt=dt, md_substeps=sub,
                                    tau_lb=dt * sub)
            E = _energy_series(run_one, p, x0, v0, n_lb)
            e = E - E[0]
            k = len(e) // 10
            per.append((float(np.std(e)), float(np.mean(e[-k:]) - np.mean(e[:k])), float(np.max(np.abs(e)))))
        out.append((per, 0.5 * float(np.sum(v0 * v0))))
    return out


def _summary(res):
    """Pooled fluctuation ratio (dt against dt/2), and the largest drift and
    excursion at dt relative to the initial kinetic energy."""
    s1 = np.array([r[0][0][0] for r in res])
    s2 = np.array([r[0][1][0] for r in res])
    ratio = float(np.sqrt(np.mean(s1 ** 2) / np.mean(s2 ** 2)))
    drift = max(abs(r[0][0][1]) / r[1] for r in res)
    excursion = max(r[0][0][2] / r[1] for r in res)
    return ratio, drift, excursion


def _passes(res):
    ratio, drift, excursion = _summary(res)
    if not np.all(np.isfinite([ratio, drift, excursion])):
        return False
    return 3.0 < ratio < 5.0 and drift < 0.01 and excursion < 0.05


def _oracle_runner(orc):
    def run_one(p, x0, v0):
        L = p["L"]
        w = orc.tables()[1]
        st = orc.State(orc.make_box(**p), w[:, None, None, None] * np.ones((19, L, L, L)), x0)
        st.v[:] = v0
        return st
    return run_one


def test_free_chain_energy_is_second_order_without_drift(orc):
    res = _verlet_check(_oracle_runner(orc))
    ratio, drift, excursion = _summary(res)
    assert 3.0 < ratio < 5.0, (ratio, res)
    assert drift < 0.01 and excursion < 0.05, (drift, excursion, res)
    assert _passes(res)


# ---------------------------------------------------------- planted copies --
_DRIFT = """        for (int b = 0; b < N; b++)
            for (int a = 0; a < 3; a++) {
                v[3 * b + a] += f[3 * b + a] / m * (0.5 * dt);
                x[3 * b + a] += v[3 * b + a] * dt;
            }
        for (int b = 0; b < N; b++) conservative_force<T>(p, x, b, &Fc[3 * b]);
"""
_KICK2 = "                v[3 * b + a] += f[3 * b + a] / m * (0.5 * dt);\n            }\n            for (int c = 0; c < 8; c++)"
_PLANTS = {
    # the conservative force evaluated at the positions before the drift
    "force_before_drift": [(_DRIFT, """        for (int b = 0; b < N; b++) conservative_force<T>(p, x, b, &Fc[3 * b]);
        for (int b = 0; b < N; b++)
            for (int a = 0; a < 3; a++) {
                v[3 * b + a] += f[3 * b + a] / m * (0.5 * dt);
                x[3 * b + a] += v[3 * b + a] * dt;
            }
""")],
    # first order (symplectic Euler): drift, then one full kick with the new force
    "single_kick": [(_DRIFT, """        for (int b = 0; b < N; b++)
            for (int a = 0; a < 3; a++) x[3 * b + a] += v[3 * b + a] * dt;
        for (int b = 0; b < N; b++) conservative_force<T>(p, x, b, &Fc[3 * b]);
"""), (_KICK2, _KICK2.replace("(0.5 * dt)", "dt"))],
}


def _planted_runner(orc, tmp_path, name):
    src = open(ORACLE_SRC).read()
    for a, b in _PLANTS[name]:
        assert src.count(a) == 1, "the oracle's substep text changed; update the planted copies"
        src = src.replace(a, b)
    path = tmp_path / f"orc_{name}.cpp"
    path.write_text(src)
    so = tmp_path / f"liborc_{name}.so"
    subprocess.run(["g++", "-O2", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                    "-o", str(so), str(path), "-lm"], check=True)
    lib = ctypes.CDLL(str(so))
    dp = ctypes.POINTER(ctypes.c_double)
    bp = ctypes.POINTER(orc.Box)
    lib.orc_run.argtypes = [bp, dp, dp, dp, dp, dp, ctypes.c_uint32, ctypes.c_int32, dp]
    lib.orc_initial_forces.argtypes = [bp, dp, dp]

    def ptr(a):
        return a.ctypes.data_as(dp)

    class St:
        def __init__(self, p, x0, v0):
            L = p["L"]
            self.box = orc.make_box(**p)
            self.n = np.ascontiguousarray(orc.tables()[1][:, None, None, None] * np.ones((19, L, L, L)))
            self.x, self.v = x0.copy(), v0.copy()
            self.f, self.fc = np.zeros_like(x0), np.zeros_like(x0)
            lib.orc_initial_forces(ctypes.byref(self.box), ptr(self.x), ptr(self.f))
            self.t = 0

        def run(self, k):
            lib.orc_run(ctypes.byref(self.box), ptr(self.n), ptr(self.x), ptr(self.v), ptr(self.f),
                        ptr(self.fc), self.t, k, None)
            self.t += k

    return lambda p, x0, v0: St(p, x0, v0)


@pytest.mark.parametrize("name", sorted(_PLANTS))
def test_planted_substep_mistakes_fail_the_energy_pin(orc, tmp_path, name):
    with np.errstate(all="ignore"):
        res = _verlet_check(_planted_runner(orc, tmp_path, name))
    assert not _passes(res), (_summary(res), res)


# ------------------------------------------------ negative populations --
def test_negative_population_count_on_hand_made_states(orc):
    """Sec. II.E: the count of n_i < 0.  A rest state with a known set of
    populations made negative; zeros of either sign are not negative, the
    smallest negative double is."""
    L = 5
    c, w, e, b = orc.tables()
    p = lbinputs.box_params("plain16", L=L, N=0)
    n = w[:, None, None, None] * p["rho0"] * np.ones((19, L, L, L))
    rng = np.random.default_rng(11)
    flat = n.reshape(-1)
    idx = rng.choice(flat.size, size=37, replace=False)
    flat[idx[:30]] = -rng.uniform(1e-6, 0.02, size=30)
    flat[idx[30]] = -5e-324
    flat[idx[31:34]] = 0.0
    flat[idx[34:]] = -0.0
    st = orc.State(orc.make_box(**p), n)
    obs = st.observables()
    assert obs[orc.OBS["neg"]] == 31.0
    # the same populations with all signs flipped up: no negative left
    st2 = orc.State(orc.make_box(**p), np.abs(n))
    assert st2.observables()[orc.OBS["neg"]] == 0.0


def test_negative_population_count_after_steps_at_paper_temperature(orc):
    """At the paper's parameters (Sec. II.E, kT = 1.2 at rho = 0.864) the
    thermal noise drives some populations negative; the oracle's count equals
    a direct count over the exported populations, and is a small fraction."""
    p = lbinputs.box_params("paper", L=6, N=0)
    c, w, e, b = orc.tables()
    L = 6
    st = orc.State(orc.make_box(**p), w[:, None, None, None] * p["rho0"] * np.ones((19, L, L, L)))
    seen = 0
    for _ in range(20):
        st.run(1)
        cnt = st.observables()[orc.OBS["neg"]]
        assert cnt == float(np.count_nonzero(st.n < 0.0))
        seen += cnt
    assert 0 < seen < 0.05 * 20 * 19 * L ** 3
