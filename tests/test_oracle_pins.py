"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the passage it follows.  None of them re-types an oracle
formula: they use exact identities, a second numpy formulation (brute.py),
the published Philox known-answer vectors and an independent library source
(rocRAND), closed-form hydrodynamics (shear and sound damping), statistical
mechanics (equipartition) and finite differences of the paper's potentials.
"""
from __future__ import annotations

import os
import shutil
import subprocess
from fractions import Fraction

import numpy as np
import pytest

import lbinputs
from oracle import brute

HERE = os.path.dirname(os.path.abspath(__file__))


def mkbox(orc, **kw):
    p = lbinputs.box_params("plain16", **kw)
    return orc.make_box(**p), p


# ------------------------------------------------------------------ Philox --
def test_philox_known_answers(orc):
    """Published Random123 known-answer vectors for Philox4x32-10."""
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "philox_kat.txt")) if l[0] != "#"]
    assert len(rows) == 3
    for r in rows:
        v = [int(s, 16) for s in r]
        got = orc.philox4x32_10(v[0:4], v[4:6])
        assert list(got) == v[6:10]
        # the numpy generator of the brute-force step agrees too
        nb = brute.philox(v[0], v[1], v[2], v[3], v[4], v[5])
        assert [int(a) for a in nb] == v[6:10]


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_philox_matches_rocrand_source(orc, tmp_path):
    """Cross-check against rocRAND's Philox4x32-10 engine (host build of its header)."""
    src = tmp_path / "p.cpp"
    src.write_text(
        "#include <rocrand/rocrand_philox4x32_10.h>\n#include <cstdio>\n#include <cstdlib>\n"
        "int main(int c, char** v){unsigned a[6];for(int i=0;i<6;i++)a[i]=strtoul(v[i+1],0,0);\n"
        "unsigned long long seed=a[0]|((unsigned long long)a[1]<<32);\n"
        "unsigned long long sub=a[4]|((unsigned long long)a[5]<<32);\n"
        "unsigned long long off=(a[2]|((unsigned long long)a[3]<<32))*4ull;\n"
        "rocrand_device::philox4x32_10_engine e(seed,sub,off);\n"
        "for(int i=0;i<4;i++)printf(\"%u \",e());printf(\"\\n\");}\n")
    exe = tmp_path / "p"
    subprocess.run(["hipcc", "-O1", "-o", str(exe), str(src)], check=True, capture_output=True)
    rng = np.random.default_rng(7)
    for _ in range(6):
        k = rng.integers(0, 2 ** 32, size=2)
        c = rng.integers(0, 2 ** 32, size=4)
        c[1] %= 2 ** 30          # rocRAND's offset argument counts words: 4 * counter must fit 64 bits
        out = subprocess.run([str(exe), *map(str, k), *map(str, c)], check=True,
                             capture_output=True, text=True).stdout.split()
        assert [int(s) for s in out] == list(orc.philox4x32_10(c, k))


def test_unit_noise_exact_and_moments(orc):
    """Word -> unit-variance uniform: odd multiples of 2^-25 scaled by sqrt(12)."""
    assert orc.unit_noise(0) == pytest.approx(np.sqrt(12) * (-(2 ** 24) + 1) * 2.0 ** -25, rel=0, abs=0)
    assert orc.unit_noise(0xFFFFFFFF) == -orc.unit_noise(0)
    vals = np.array([orc.unit_noise(int(w)) for w in np.linspace(0, 2 ** 32 - 1, 4097).astype(np.uint64)])
    assert abs(vals.mean()) < 1e-3 and abs((vals ** 2).mean() - 1.0) < 2e-3


# ----------------------------------------------------------- D3Q19 tables --
def test_weight_identities(orc):
    """Sec. II.B: w = 1/3, 1/18, 1/36 and c_s^2 = 1/3: sum w = 1, sum w c = 0,
    sum w c_a c_b = delta/3, fourth moment isotropic (needed for the
    Navier-Stokes limit of the second-order equilibrium)."""
    c, w, e, b = orc.tables()
    F = [Fraction(x).limit_denominator(100) for x in w]
    assert sum(F) == 1
    for a in range(3):
        assert sum(Fraction(int(c[i, a])) * F[i] for i in range(19)) == 0
        for bb in range(3):
            s = sum(Fraction(int(c[i, a] * c[i, bb])) * F[i] for i in range(19))
            assert s == (Fraction(1, 3) if a == bb else 0)
    d = np.eye(3)
    for a in range(3):
        for bb in range(3):
            for cc in range(3):
                for dd in range(3):
                    s = sum(w[i] * c[i, a] * c[i, bb] * c[i, cc] * c[i, dd] for i in range(19))
                    iso = (d[a, bb] * d[cc, dd] + d[a, cc] * d[bb, dd] + d[a, dd] * d[bb, cc]) / 9
                    assert abs(s - iso) < 1e-15
    # velocity magnitudes 0, 1, sqrt 2 with multiplicities 1, 6, 12
    mags = sorted((c * c).sum(1).astype(int).tolist())
    assert mags == [0] + [1] * 6 + [2] * 12
    assert len({tuple(v) for v in c.astype(int)}) == 19


def test_mode_basis_orthogonal_and_norms(orc):
    """The 19 modes are orthogonal under the weights (exact rationals) and span
    mass, momentum, the six stress components and nine ghosts."""
    c, w, e, b = orc.tables()
    Fw = [Fraction(x).limit_denominator(100) for x in w]
    E = [[Fraction(int(round(v))) for v in row] for row in e]
    assert all(abs(e[k, i] - round(e[k, i])) == 0 for k in range(19) for i in range(19))
    for k in range(19):
        for l in range(19):
            s = sum(Fw[i] * E[k][i] * E[l][i] for i in range(19))
            if k != l:
                assert s == 0, (k, l)
    gold = open(os.path.join(HERE, "golden", "mode_norms.txt")).read().split("\n")
    gold = [l for l in gold if l and l[0] != "#"][0].split()
    for k in range(19):
        assert Fraction(b[k]).limit_denominator(100) == Fraction(gold[k])
    # modes 0..9 span {1, c_a, c_a c_b}: the hydrodynamic moments
    hyd = [np.ones(19)] + [c[:, a] for a in range(3)] + \
          [c[:, a] * c[:, bb] for a in range(3) for bb in range(a, 3)]
    H = np.array(hyd)
    P = e[:10]
    assert np.linalg.matrix_rank(np.vstack([H, P])) == 10
    assert np.linalg.matrix_rank(e) == 19
    assert int(np.count_nonzero(e)) == 207


# ------------------------------------------------------------- collision --
def _rand_state(orc, L, amp, seed, rho0=1.0):
    c, w, e, b = orc.tables()
    d = lbinputs.random_deviations(L, amp, seed)
    return w[:, None, None, None] * rho0 * (1.0 + d)


def test_relaxed_collision_gives_paper_equilibrium(orc):
    """With every rate 1 and no noise the collision returns exactly the
    second-order equilibrium of Sec. II.B evaluated at (rho, u) of the node."""
    bx, p = mkbox(orc, L=4, N=0, kT=0.0)
    c, w, e, b = orc.tables()
    rng = np.random.default_rng(3)
    for _ in range(20):
        n = w * (1 + rng.uniform(-0.3, 0.3, size=19))
        out = orc.collide_one(bx, n)
        rho = n.sum()
        u = (c.T @ n) / rho
        ref = brute.equilibrium(np.array([rho]), u[:, None])[:, 0]
        np.testing.assert_allclose(out, ref, rtol=0, atol=2e-16)


@pytest.mark.parametrize("L", [2, 3])
@pytest.mark.parametrize("therm", [2, 1, 0])
def test_brute_force_tiny_lattice(orc, L, therm):
    """Independent numpy statement of one collide+stream step (dense 19x19
    inverse, population-space equilibrium and forcing, explicit permutation
    streaming, its own Philox) agrees with the C oracle to round-off."""
    bx, p = mkbox(orc, L=L, N=0, kT=0.3, omega_s=1.3, omega_b=0.7, omega_g=1.6,
                  therm=therm, seed=11, box_id=5)
    n = _rand_state(orc, L, 0.2, 1)
    dp = lbinputs.random_impulses(L, 0.01, 2)
    st = orc.State(bx, n)
    st.t = 17
    st.collide_stream(dp)
    ref = brute.step(n, dp, p, 17)
    np.testing.assert_allclose(st.n, ref, rtol=0, atol=5e-15)


def test_streaming_is_permutation():
    brute.all_permutation_check(3)


def test_conservation_mass_momentum(orc):
    """Collision conserves rho and j (Sec. II.B); streaming permutes: total
    mass and momentum are invariant with full noise and non-unit rates; an
    impulse field adds exactly its own sum to the momentum."""
    L = 6
    bx, p = mkbox(orc, L=L, N=0, kT=0.05, omega_s=1.4, omega_b=0.9, omega_g=1.2)
    c, w, e, b = orc.tables()
    st = orc.State(bx, _rand_state(orc, L, 0.1, 4))
    o0 = st.observables()
    st.run(20)
    o1 = st.observables()
    assert abs(o1[0] - o0[0]) / o0[0] < 1e-13
    np.testing.assert_allclose(o1[1:4], o0[1:4], atol=1e-12)
    dp = lbinputs.random_impulses(L, 1e-3, 9, density=0.1)
    st.collide_stream(dp)
    o2 = st.observables()
    np.testing.assert_allclose(o2[1:4] - o1[1:4], dp.reshape(3, -1).sum(1), atol=1e-12)
    assert abs(o2[0] - o0[0]) / o0[0] < 1e-13


def test_equilibrium_fixed_point(orc):
    """kT = 0: a uniform n^eq(rho0, u0) is a fixed point of collide+stream."""
    L = 5
    bx, p = mkbox(orc, L=L, N=0, kT=0.0, omega_s=1.3, omega_b=0.7, omega_g=1.5)
    V = L ** 3
    u0 = np.array([0.02, -0.01, 0.015])
    n = brute.equilibrium(np.full(V, 1.0), np.repeat(u0[:, None], V, 1)).reshape(19, L, L, L)
    st = orc.State(bx, n)
    st.run(10)
    np.testing.assert_allclose(st.n, n, rtol=0, atol=4e-15)   # ten steps of FP64 round-off


def test_shear_wave_decay_sets_viscosity(orc):
    """Transverse wave u_x(z) decays as exp(-nu k^2 t), nu = c_s^2 (1/omega_s - 1/2)."""
    L = 32
    V = L ** 3
    c, w, e, b = orc.tables()
    z = np.arange(L)
    k = 2 * np.pi / L
    for ws in (1.25, 0.8):
        bx, p = mkbox(orc, L=L, N=0, kT=0.0, omega_s=ws)
        u = np.zeros((3, L, L, L))
        u[0] = 1e-4 * np.sin(k * z)[:, None, None]
        st = orc.State(bx, brute.equilibrium(np.ones(V), u.reshape(3, -1)).reshape(19, L, L, L))

        def amp():
            jx = np.tensordot(c[:, 0], st.n, axes=(0, 0))
            return np.sum(jx * np.sin(k * z)[:, None, None])

        st.run(20)
        a1 = amp()
        st.run(80)
        a2 = amp()
        nu = -np.log(a2 / a1) / (k * k * 80)
        assert nu == pytest.approx((1 / 3) * (1 / ws - 0.5), rel=5e-3)


def test_sound_damping_sets_bulk_viscosity(orc):
    """Longitudinal wave energy decays as exp(-(4 nu/3 + nu_b) k^2 t) with
    nu_b = (2/3) c_s^2 (1/omega_b - 1/2): pins the bulk mode and its rate."""
    L = 32
    V = L ** 3
    c, w, e, b = orc.tables()
    x = np.arange(L)
    k = 2 * np.pi / L
    for wb in (0.6, 1.5):
        bx, p = mkbox(orc, L=L, N=0, kT=0.0, omega_s=1.0, omega_b=wb)
        rho = np.broadcast_to((1 + 1e-4 * np.cos(k * x))[None, None, :], (L, L, L)).reshape(-1)
        st = orc.State(bx, brute.equilibrium(rho, np.zeros((3, V))).reshape(19, L, L, L))
        ts, Es = [], []
        for t in range(0, 331, 2):
            dr = st.n.sum(0) - 1.0
            jx = np.tensordot(c[:, 0], st.n, axes=(0, 0))
            rh = 2.0 / V * np.sum(dr * np.cos(k * x)[None, None, :])
            jh = 2.0 / V * np.sum(jx * np.sin(k * x)[None, None, :])
            ts.append(t)
            Es.append(rh * rh / 3 + jh * jh)
            st.run(2)
        D = -np.polyfit(ts, np.log(Es), 1)[0] / (k * k)
        nu, nub = (1 / 3) * 0.5, (2 / 3) * (1 / 3) * (1 / wb - 0.5)
        assert D == pytest.approx(4 * nu / 3 + nub, rel=1.5e-2)


@pytest.mark.parametrize("omegas", [(1.0, 1.0, 1.0), (1.25, 0.8, 1.4)])
def test_equipartition_of_modes(orc, omegas):
    """Sec. II.B: with all non-conserved modes thermalized every mode k >= 4
    fluctuates with <m_k^2> = mu rho0 b_k (mu = kT/c_s^2 in lattice units),
    at unit and at non-unit relaxation rates."""
    L = 12
    ws, wb, wg = omegas
    kT = 1e-2   # MD units; kT_lat = 1e-4
    bx, p = mkbox(orc, L=L, N=0, kT=kT, omega_s=ws, omega_b=wb, omega_g=wg, therm=2)
    c, w, e, b = orc.tables()
    st = orc.State(bx, (w[:, None, None, None] * np.ones((19, L, L, L))))
    st.run(30)
    acc = np.zeros(19)
    n_s = 120
    for _ in range(n_s):
        st.run(1)
        acc += st.observables()[19:38]
    var = acc / (n_s * L ** 3)
    mu = 3 * kT * p["tau_lb"] ** 2
    ratio = var / (mu * 1.0 * b)
    np.testing.assert_allclose(ratio[4:], 1.0, atol=0.025)


def test_stress_only_thermalization_flag(orc):
    """Sec. II.B: the original scheme puts noise on the stress modes only.
    Post-collision ghosts then carry no noise (gamma_g m exactly); with full
    thermalization they do; with none the collision is deterministic."""
    c, w, e, b = orc.tables()
    rng = np.random.default_rng(5)
    n = w * (1 + rng.uniform(-0.2, 0.2, size=19))
    m = e @ n
    for wg in (1.0, 1.3):
        outs = {}
        for therm in (0, 1, 2):
            bx, p = mkbox(orc, L=4, N=0, kT=0.5, omega_s=1.2, omega_b=0.9, omega_g=wg, therm=therm)
            outs[therm] = e @ orc.collide_one(bx, n, r=3, t=9)
        bx0, _ = mkbox(orc, L=4, N=0, kT=0.0, omega_s=1.2, omega_b=0.9, omega_g=wg)
        det = e @ orc.collide_one(bx0, n, r=3, t=9)
        np.testing.assert_allclose(outs[0], det, atol=1e-15)
        np.testing.assert_allclose(outs[1][10:], (1 - wg) * m[10:], atol=1e-15)
        np.testing.assert_allclose(outs[1][:10], outs[2][:10], atol=1e-15)
        assert np.all(np.abs(outs[1][4:10] - det[4:10]) > 1e-6)
        assert np.all(np.abs(outs[2][10:] - det[10:]) > 1e-6)


def test_stress_only_thermalization_is_poor_at_short_scales(orc):
    """Sec. II.B: thermalizing only the stress modes is correct in the
    hydrodynamic limit but not at the lattice scale: node-level stress-mode
    variances fall well short of mu rho0 b_k, while full thermalization meets it."""
    L = 10
    kT = 1e-2
    c, w, e, b = orc.tables()
    res = {}
    for therm in (1, 2):
        bx, p = mkbox(orc, L=L, N=0, kT=kT, therm=therm)
        st = orc.State(bx, (w[:, None, None, None] * np.ones((19, L, L, L))))
        st.run(20)
        acc = np.zeros(19)
        for _ in range(60):
            st.run(1)
            acc += st.observables()[19:38]
        res[therm] = acc / (60 * L ** 3) / (3 * kT * p["tau_lb"] ** 2 * b)
    assert np.all(np.abs(res[2][4:10] - 1) < 0.04)
    assert np.all(res[1][4:10] < 0.8)


# -------------------------------------------------------------- chain / MD --
def _fene_wca_energy(p, x):
    """Total potential of Sec. II.A (FENE on the bonds along each chain, LJ cut
    and shifted at 2^(1/6) sigma between all pairs, minimum image)."""
    N, L = len(x), p["L"]
    n = p.get("chain_len", 0) or N
    U = 0.0
    for i in range(N - 1):
        if (i + 1) % n == 0:      # last bead of a chain: no bond to the next chain
            continue
        r2 = np.sum((x[i + 1] - x[i]) ** 2)
        U += -0.5 * p["k_fene"] * p["r0_fene"] ** 2 * np.log(1 - r2 / p["r0_fene"] ** 2)
    for i in range(N):
        for j in range(i + 1, N):
            d = x[i] - x[j]
            d -= L * np.round(d / L)
            r = np.sqrt(np.sum(d * d))
            if r <= 2 ** (1 / 6) * p["sigma_wca"]:
                sr6 = (p["sigma_wca"] / r) ** 6
                U += 4 * p["eps_wca"] * (sr6 * sr6 - sr6 + 0.25)
    return U


def test_forces_are_minus_gradient(orc):
    bx, p = mkbox(orc, L=8, N=6)
    # tight zig-zag: pairs (0,2), (1,3), ... sit inside the LJ cut-off, bonds below R0
    ang = np.deg2rad(62.0)
    x = np.array([[0.0, 0, 0], [0.97, 0, 0], [0.97 - 0.95 * np.cos(ang), 0.95 * np.sin(ang), 0.1],
                  [1.9, 0.9, -0.1], [1.2, 1.6, 0.3], [2.1, 1.9, 0.2]]) + 3.0
    F = orc.initial_forces(bx, x)
    h = 1e-6
    for bead in range(6):
        for a in range(3):
            xp, xm = x.copy(), x.copy()
            xp[bead, a] += h
            xm[bead, a] -= h
            g = (_fene_wca_energy(p, xp) - _fene_wca_energy(p, xm)) / (2 * h)
            assert F[bead, a] == pytest.approx(-g, rel=1e-6, abs=1e-6)


def test_several_chains_forces_are_minus_gradient(orc):
    """Three chains of three beads (Sec. III.C's semidilute solution): bonds
    only along each chain, LJ between all beads.  The end of each chain sits
    inside the LJ range of the next chain's start, so both a bond wrongly
    carried across chains and a missing inter-chain LJ term change the force."""
    bx, p = mkbox(orc, L=8, N=9, chain_len=3)
    x = np.array([[2.0, 2.0, 2.0], [2.97, 2.0, 2.0], [3.5, 2.8, 2.1],
                  [4.0, 3.7, 2.0], [4.9, 4.0, 2.2], [5.2, 4.9, 2.6],
                  [6.1, 5.3, 2.9], [6.6, 6.1, 3.0], [7.5, 6.4, 3.3]])
    r_end_start = [np.linalg.norm(x[3 * c + 2] - x[3 * c + 3]) for c in range(2)]
    assert max(r_end_start) < 2 ** (1 / 6) and min(r_end_start) > 0.8
    F = orc.initial_forces(bx, x)
    h = 1e-6
    for bead in range(9):
        for a in range(3):
            xp, xm = x.copy(), x.copy()
            xp[bead, a] += h
            xm[bead, a] -= h
            g = (_fene_wca_energy(p, xp) - _fene_wca_energy(p, xm)) / (2 * h)
            assert F[bead, a] == pytest.approx(-g, rel=1e-6, abs=1e-6)
    # chain_len = N is the single chain of the default
    b1, _ = mkbox(orc, L=8, N=9, chain_len=9)
    b0, _ = mkbox(orc, L=8, N=9, chain_len=0)
    assert np.array_equal(orc.initial_forces(b1, x), orc.initial_forces(b0, x))


def test_separated_chains_move_as_single_chains(orc):
    """Without friction and noise (zeta = 0, kT = 0) chains further apart than
    the LJ range do not see each other or the fluid: each follows the
    trajectory it has alone in the box, bit for bit (the LJ terms of the other
    chains are zero and skipped)."""
    L, n, M = 16, 5, 3
    ang = np.deg2rad(70.0)
    one = np.array([[0.0, 0, 0], [0.97, 0, 0], [0.97 + 0.9 * np.cos(ang), 0.9 * np.sin(ang), 0.2],
                    [0.5, 1.5, 0.1], [-0.3, 1.2, -0.4]])
    offs = [np.array([3.0, 4.0, 8.0]), np.array([8.0, 9.0, 8.0]), np.array([13.0, 3.0, 2.0])]
    x = np.concatenate([one + o for o in offs])
    kw = dict(L=L, kT=0.0, zeta=0.0, k_fene=7.0, r0_fene=2.0)
    bx, p = mkbox(orc, N=n * M, chain_len=n, **kw)
    n0 = np.ones((19, L, L, L)) * orc.tables()[1][:, None, None, None]
    st = orc.State(bx, n0, x)
    st.run(20)
    moved = 0.0
    for c in range(M):
        b1, _ = mkbox(orc, N=n, **kw)
        one_st = orc.State(b1, n0, x[c * n:(c + 1) * n])
        one_st.run(20)
        assert np.array_equal(st.x[c * n:(c + 1) * n], one_st.x)
        assert np.array_equal(st.v[c * n:(c + 1) * n], one_st.v)
        moved = max(moved, float(np.max(np.abs(one_st.x - x[c * n:(c + 1) * n]))))
    assert moved > 1e-3
    # and the chains stayed out of each other's LJ range
    d = st.x[:, None] - st.x[None]
    d -= L * np.round(d / L)
    r = np.sqrt(np.sum(d * d, -1))
    for c in range(M):
        r[c * n:(c + 1) * n, c * n:(c + 1) * n] = 99.0
    assert r.min() > 2 ** (1 / 6)


def test_wca_vanishes_at_cutoff_and_min_image(orc):
    bx, p = mkbox(orc, L=8, N=3, k_fene=0.0)
    rc = 2 ** (1 / 6)
    x = np.array([[1.0, 1, 1], [5.0, 5, 5], [1.0 + rc * (1 - 1e-9), 1, 1]])
    F = orc.initial_forces(bx, x)
    assert abs(F[2, 0]) < 1e-6 and abs(F[0, 0]) < 1e-6
    x[2, 0] = 1.0 + rc * (1 + 1e-9)
    assert np.all(orc.initial_forces(bx, x) == 0.0)
    x2 = np.array([[0.2, 4, 4], [4.0, 4, 4], [7.6, 4, 4]])   # 0.2 and 7.6 are 0.6 apart through the wall
    bx3, p3 = mkbox(orc, L=8, N=3, k_fene=0.0)
    F2 = orc.initial_forces(bx3, x2)
    assert F2[0, 0] > 0 and F2[2, 0] < 0 and F2[0, 0] == pytest.approx(-F2[2, 0], rel=1e-12)


def test_linear_field_interpolated_exactly(orc):
    """Trilinear weights reproduce a linear velocity field exactly (one substep,
    bead at rest, no noise: v = zeta u_b dt / 2m)."""
    L = 8
    bx, p = mkbox(orc, L=L, N=1, kT=0.0, md_substeps=1, tau_lb=0.01)
    V = L ** 3
    z, y, x = np.meshgrid(np.arange(L), np.arange(L), np.arange(L), indexing="ij")
    a0, g = np.array([0.01, -0.02, 0.005]), np.array([[0.002, 0.001, -0.003]] * 3) * np.array([[1], [2], [3]])
    u_md = a0[:, None] + g @ np.array([x.reshape(-1), y.reshape(-1), z.reshape(-1)])
    n = brute.equilibrium(np.ones(V), u_md * p["tau_lb"]).reshape(19, L, L, L)
    bead = np.array([[3.3, 4.7, 2.25]])
    st = orc.State(bx, n, bead)
    st.couple()
    ub = 2 * p["mass"] * st.v[0] / (p["zeta"] * p["md_dt"])
    np.testing.assert_allclose(ub, a0 + g @ bead[0], rtol=1e-12)


def test_coupling_conserves_total_momentum(orc):
    """Sec. II.B: the fluid receives exactly the momentum the beads lose to
    friction and noise.  At LB-step boundaries
    P_fluid + P_beads + (dt/2) sum F_coupling(last substep) is invariant."""
    L, N = 10, 8
    bx, p = mkbox(orc, L=L, N=N, kT=0.05)
    c, w, e, b = orc.tables()
    st = orc.State(bx, _rand_state(orc, L, 0.02, 5), lbinputs.saw_chain(N, L, 5))
    st.v[:] = np.random.default_rng(1).normal(scale=0.3, size=st.v.shape)
    o0 = st.observables()
    st.run(15)
    o1 = st.observables()
    np.testing.assert_allclose(o1[10:13], o0[10:13], atol=1e-11)
    assert np.max(np.abs(o1[7:10] - o0[7:10])) > 1e-3      # momentum did move between beads and fluid


def test_chain_observables_closed_forms(orc):
    """R_g^2 by the pair formula of Sec. III.A equals the centre-of-mass form;
    R_e^2 is the end-to-end square."""
    bx, p = mkbox(orc, L=8, N=7)
    x = lbinputs.saw_chain(7, 8, 9)
    st = orc.State(bx, np.ones((19, 8, 8, 8)) / 19, x)
    o = st.observables()
    com = x.mean(0)
    np.testing.assert_allclose(o[13:16], com, rtol=1e-14)
    assert o[16] == pytest.approx(np.mean(np.sum((x - com) ** 2, 1)), rel=1e-13)
    assert o[17] == pytest.approx(np.sum((x[-1] - x[0]) ** 2), rel=1e-14)


def test_several_chains_observables_closed_forms(orc):
    """M straight rods of n beads with spacings a_c: R_g^2 = a_c^2 (n^2 - 1) / 12
    and R_e^2 = a_c^2 (n - 1)^2 per rod; the box reports their means over the
    chains, and the centre of mass of all beads."""
    n, M = 6, 4
    a = np.array([0.9, 1.0, 0.75, 1.2])
    rods = []
    for c in range(M):
        r = np.zeros((n, 3))
        r[:, c % 3] = a[c] * np.arange(n)
        rods.append(r + [1.0 + c, 2.0 * c, 0.5])
    x = np.concatenate(rods)
    bx, p = mkbox(orc, L=12, N=n * M, chain_len=n)
    st = orc.State(bx, np.ones((19, 12, 12, 12)) / 19, x)
    o = st.observables()
    assert o[16] == pytest.approx(np.mean(a ** 2) * (n * n - 1) / 12, rel=1e-13)
    assert o[17] == pytest.approx(np.mean(a ** 2) * (n - 1) ** 2, rel=1e-13)
    np.testing.assert_allclose(o[13:16], x.mean(0), rtol=1e-14)


@pytest.mark.slow
def test_bead_equipartition(orc):
    """Fluctuation-dissipation (Sec. II.B): a bead in the thermal fluid reaches
    <m v_a^2> = kT per component when the fluid moves little during one LB
    step of frozen-field substeps (zeta tau_lb / m = 0.2).  At the standard
    workloads' zeta tau_lb / m = 2 the frozen-field substeps run about 20%
    hot; that is a property of the time discretisation, recorded in the
    design notes, not of the noise amplitude pinned here."""
    L = 6
    kT = 1e-2
    bx, p = mkbox(orc, L=L, N=1, kT=kT, zeta=2.0)
    c, w, e, b = orc.tables()
    st = orc.State(bx, w[:, None, None, None] * np.ones((19, L, L, L)), np.array([[2.5, 3.1, 1.7]]))
    st.run(300)
    h = st.run(6000, record_velocities=True)
    v2 = np.mean(h[:, 0, :] ** 2) * p["mass"]
    assert v2 == pytest.approx(kT, rel=0.04)


# ---------------------------------------------------------- window tangent --
def test_window_tangent_values_equal_run(orc):
    """The dual-number instantiation performs the same value arithmetic."""
    L, N = 6, 4
    bx, p = mkbox(orc, L=L, N=N, kT=1e-2, omega_s=1.2, omega_b=0.9)
    n0 = _rand_state(orc, L, 0.02, 7)
    x0 = lbinputs.saw_chain(N, L, 7)
    a = orc.State(bx, n0, x0)
    b = a.copy()
    h = a.run(6, record_velocities=True)
    hv, dh = b.window_tangent(6)
    assert np.array_equal(h, hv) and np.array_equal(a.n, b.n) and np.array_equal(a.x, b.x)


@pytest.mark.parametrize("N,chain_len", [(4, 0), (6, 3)])
def test_window_tangent_matches_finite_differences(orc, N, chain_len):
    """d v(t) / d(omega_shear, omega_bulk, zeta) by forward mode equals central
    differences of the oracle's own window (one chain, and two chains)."""
    L, T = 6, 8
    base = dict(L=L, N=N, chain_len=chain_len, kT=1e-2, omega_s=1.2, omega_b=0.9, zeta=20.0)
    n0 = _rand_state(orc, L, 0.02, 8)
    x0 = lbinputs.initial_chains(dict(L=L, N=N, chain_len=chain_len, seed=8))
    bx, p = mkbox(orc, **base)
    _, dh = orc.State(bx, n0, x0).window_tangent(T)
    for k, name in enumerate(("omega_s", "omega_b", "zeta")):
        hstep = 1e-6 * base[name]
        res = []
        for sgn in (+1, -1):
            kw = dict(base)
            kw[name] = base[name] + sgn * hstep
            b2, _ = mkbox(orc, **kw)
            res.append(orc.State(b2, n0, x0).run(T, record_velocities=True))
        fd = (res[0] - res[1]) / (2 * hstep)
        scale = np.max(np.abs(fd))
        assert scale > 0
        np.testing.assert_allclose(dh[..., k], fd, rtol=0, atol=1e-5 * scale)
