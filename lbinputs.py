"""Seeded synthetic inputs shared by the GPU library's callers and the oracle.

This module holds input generation only: parameter presets, the initial chain
and the batched box table.  It contains none of the method's arithmetic, so
the GPU path and the oracle can both take their inputs from here without
sharing any of the computation under test.

Workload recipe (the paper uses no public dataset; its runs are synthetic
single-chain boxes, Sec. II.E "Choice of parameters" and Sec. III.C):
  * fluid: cubic periodic box of L^3 nodes, lattice spacing 1 (one LJ sigma),
    uniform rest state n_i = w_i rho0;
  * chain: N beads, self-avoiding random walk of bond 0.97 sigma started at the
    box centre, directions uniform on the sphere, a step rejected if it comes
    closer than 0.9 sigma to any earlier bead, velocities zero;
  * batched sweep: L drawn uniformly from {16,24,32,48,64}, N uniformly from
    {8,16,32,64} restricted to N <= L;
  * several chains in one box (semidilute solution, Sec. III.C): M walks of n
    beads, each started at a uniform random point, every bead kept 0.9 sigma
    from all beads placed before it.
"""
from __future__ import annotations

import numpy as np

# Fluid and chain parameters of the standard workloads.  Units: chain in LJ
# units (sigma = m = eps = 1), lattice spacing 1 sigma, LB step tau_lb =
# md_substeps * md_dt, rho0 in m / sigma^3, kT in eps.
BASE = dict(rho0=1.0, omega_s=1.0, omega_b=1.0, omega_g=1.0, kT=1e-4, therm=2,
            tau_lb=0.1, md_dt=0.01, md_substeps=10, mass=1.0, zeta=20.0,
            k_fene=30.0, r0_fene=1.5, eps_wca=1.0, sigma_wca=1.0, seed=1, box_id=0,
            chain_len=0)

PRESETS = {
    # 16^3, FP64, N=16, 1000 steps
    "plain16": dict(BASE, L=16, N=16, steps=1000, precision="fp64"),
    # 64^3, FP32 deviation storage, N=64, 10000 steps
    "single64": dict(BASE, L=64, N=64, steps=10000, precision="fp32"),
    # 256 boxes of uneven L and N, FP32, 5000 steps
    "batched256": dict(BASE, n_boxes=256, steps=5000, precision="fp32"),
    # 256^3, N=1024, FP32, 2000 steps
    "prec256": dict(BASE, L=256, N=1024, steps=2000, precision="fp32"),
    # 32^3, N=32, 200-step adjoint window, checkpoints every 20 steps
    "adjoint32": dict(BASE, L=32, N=32, steps=200, checkpoint_every=20, precision="fp32"),
    # the paper's own parameter set (Sec. II.E): kT=1.2, rho=0.864, nu=2.8,
    # zeta_bare=20.8, k_FENE=7, R0=2, dt=0.01, LB step 0.02, N=32
    "paper": dict(BASE, L=15, N=32, rho0=0.864, kT=1.2, zeta=20.8, k_fene=7.0,
                  r0_fene=2.0, md_dt=0.01, md_substeps=2, tau_lb=0.02,
                  omega_s=1.0 / (3.0 * 2.8 * 0.02 + 0.5), omega_b=1.0 / (3.0 * 2.8 * 0.02 + 0.5),
                  steps=1000, precision="fp32"),
}
# semidilute solution (Sec. III.C): 32 chains of 32 beads at the paper's
# parameters in a 20^3 box, monomer concentration 0.128 / sigma^3, about the
# overlap concentration of a 32-bead chain (R_g^2 ~ 15); a batch of 64 boxes
PRESETS["semidilute"] = dict(PRESETS["paper"], L=20, N=1024, chain_len=32, n_boxes=64, steps=500,
                             precision="fp32")

BOX_FIELDS = ("L", "N", "rho0", "omega_s", "omega_b", "omega_g", "kT", "therm", "tau_lb",
              "md_dt", "md_substeps", "mass", "zeta", "k_fene", "r0_fene", "eps_wca",
              "sigma_wca", "seed", "box_id", "chain_len")


def box_params(preset: str | dict, **override) -> dict:
    p = dict(PRESETS[preset]) if isinstance(preset, str) else dict(preset)
    p.update(override)
    return {k: p[k] for k in BOX_FIELDS}


def saw_chain(N: int, L: int, seed: int, bond: float = 0.97, min_dist: float = 0.9,
              max_tries: int = 100000) -> np.ndarray:
    """Self-avoiding random walk of N beads (unwrapped coordinates), float64 (N,3)."""
    rng = np.random.default_rng([seed, N, L, 2])
    x = np.zeros((N, 3))
    if N == 0:
        return x
    x[0] = 0.5 * L
    for i in range(1, N):
        for _ in range(max_tries):
            d = rng.normal(size=3)
            d *= bond / np.linalg.norm(d)
            cand = x[i - 1] + d
            if i < 2:
                break
            diff = x[: i - 1] - cand
            diff -= L * np.round(diff / L)
            if np.min(np.einsum("ij,ij->i", diff, diff)) >= min_dist * min_dist:
                break
        else:
            raise RuntimeError("self-avoiding walk could not be grown")
        x[i] = cand
    return x


def saw_chains(M: int, n: int, L: int, seed: int, bond: float = 0.97, min_dist: float = 0.9,
               max_tries: int = 100000) -> np.ndarray:
    """M self-avoiding chains of n beads each in one periodic box, float64
    (M*n, 3), chain c at rows c*n .. c*n+n-1 (unwrapped within a chain).  Each
    chain starts at a uniform random point and grows like saw_chain; a bead is
    rejected if it comes closer than min_dist (minimum image) to any bead
    placed before it, of any chain."""
    rng = np.random.default_rng([seed, M, n, L, 6])
    x = np.zeros((M * n, 3))
    k = 0

    def clear(cand, upto):
        if upto == 0:
            return True
        diff = x[:upto] - cand
        diff -= L * np.round(diff / L)
        return np.min(np.einsum("ij,ij->i", diff, diff)) >= min_dist * min_dist

    for c in range(M):
        for i in range(n):
            for _ in range(max_tries):
                if i == 0:
                    cand = rng.uniform(0.0, L, size=3)
                    if clear(cand, k):
                        break
                    continue
                d = rng.normal(size=3)
                d *= bond / np.linalg.norm(d)
                cand = x[k - 1] + d
                if clear(cand, k):   # (the bead it is bonded to is one bond away)
                    break
            else:
                raise RuntimeError("self-avoiding chains could not be grown")
            x[k] = cand
            k += 1
    return x


def initial_chains(p: dict, seed: int | None = None) -> np.ndarray:
    """Initial beads of box p: one SAW of N beads, or N / chain_len SAWs."""
    N, L = int(p["N"]), int(p["L"])
    n = int(p.get("chain_len", 0) or N)
    s = int(p["seed"] if seed is None else seed)
    if N == 0 or n == N:
        return saw_chain(N, L, s)
    return saw_chains(N // n, n, L, s)


def batched_table(n_boxes: int = 256, seed: int = 1):
    """(L, N) per box for the finite-size sweep: L ~ U{16,24,32,48,64}, N ~ U{n <= L}."""
    rng = np.random.default_rng([seed, 3])
    Ls = rng.choice([16, 24, 32, 48, 64], size=n_boxes)
    Ns = np.array([rng.choice([n for n in (8, 16, 32, 64) if n <= L]) for L in Ls])
    return [(int(L), int(N)) for L, N in zip(Ls, Ns)]


def random_deviations(L: int, amp: float, seed: int) -> np.ndarray:
    """Uniform random numbers in [-amp, amp], shape (19, L, L, L), float64."""
    rng = np.random.default_rng([seed, L, 4])
    return rng.uniform(-amp, amp, size=(19, L, L, L))


def random_impulses(L: int, amp: float, seed: int, density: float = 1.0) -> np.ndarray:
    """Random per-node impulse field (3, L, L, L); a fraction `density` of nodes non-zero."""
    rng = np.random.default_rng([seed, L, 5])
    f = rng.uniform(-amp, amp, size=(3, L, L, L))
    if density < 1.0:
        f *= (rng.uniform(size=(1, L, L, L)) < density)
    return f
