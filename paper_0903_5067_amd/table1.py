"""A single chain of N = 32 at the paper's parameters (Sec. II.E: kT = 1.2,
rho = 0.864, nu = 2.8, zeta = 20.8, k_FENE = 7, R0 = 2, dt = 0.01, LB step
0.02) in periodic boxes of side L: the chain properties of the paper's
Table 1 (LB columns), from many independent boxes advanced together on the
GPU in one batch.

Each box has its own Philox stream (key (seed, box)) and its own starting
walk. Boxes are equilibrated, then sampled every `sample_tau` (LJ time).
Static averages and their errors come from the spread of per-box time
averages, since the boxes are independent:
  <R_e^2>, <R_g^2> (GPU FP64 sums), <1/R_H> (snapshots), nu from S(k) ~ k^(-1/nu),
dynamic ones from the sampled centre of mass and the two innermost beads:
  g1 exponent over t in [20, 80], D_CM from g3 = 6 D t over the same window
  and over [100, 1000], tau_tr = <R_g^2> / (6 D_CM), the first Rouse mode's
  autocorrelation at t = 700,
the beads' kinetic temperature <m v^2> / 3 against kT, and the fraction of
populations n_i < 0 at the samples (Sec. II.E).

    python -m paper_0903_5067_amd.table1 --L 10 15 --boxes 128 --out result.json
    python -m paper_0903_5067_amd.table1 --therm 1 ...   (stress modes only)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

# LB columns of the paper's Table 1 (N = 32; LB time step 0.02): value, error
PAPER_TABLE1 = {
    10: {"nu": (0.615, 0.005), "re2": (94.56, 1.20), "rg2": (14.83, 0.10), "inv_rh": (0.291, 0.0005),
         "g1_exponent": (0.640, 0.0005), "g3_exponent": (1.008, 0.0008),
         "d_cm": (3.914e-3, 1e-6), "tau_tr": (631.36, 4.43)},
    15: {"nu": (0.617, 0.005), "re2": (100.05, 1.26), "rg2": (15.31, 0.11), "inv_rh": (0.290, 0.0005),
         "g1_exponent": (0.675, 0.0005), "g3_exponent": (1.020, 0.0008),
         "d_cm": (5.162e-3, 1e-6), "tau_tr": (492.01, 3.56)},
    25: {"nu": (0.619, 0.005), "re2": (100.20, 1.28), "rg2": (15.36, 0.11), "inv_rh": (0.289, 0.0005),
         "g1_exponent": (0.710, 0.0005), "g3_exponent": (1.050, 0.0008),
         "d_cm": (6.959e-3, 2e-6), "tau_tr": (368.51, 2.67)},
}
# the same table's g1 exponents from LB runs that thermalize the stress modes only
PAPER_G1_STRESS_ONLY = {10: (0.645, 0.0006), 15: (0.684, 0.0006), 25: (0.714, 0.0006)}


def _say(*a):
    print("[table1]", *a, flush=True)


def run_box_size(L: int, n_boxes: int, equil_tau: float, prod_tau: float, sample_tau: float, seed: int = 1,
                 precision: int | None = None, therm: int = 2) -> dict:
    import lbinputs
    import paper_0903_5067_amd as lbm
    from paper_0903_5067_amd import analysis as an

    prec = lbm.FP32_DEV if precision is None else precision
    base = lbinputs.box_params("paper", L=L, seed=seed, therm=therm)
    boxes = [dict(base, box_id=i) for i in range(n_boxes)]
    N = int(base["N"])
    x0 = np.concatenate([lbinputs.saw_chain(N, L, seed + 7919 * i) for i in range(n_boxes)])
    tau = float(base["tau_lb"])
    every = int(round(sample_tau / tau))
    every += every & 1
    s = lbm.LBSystem(boxes, precision=prec, bead_x0=x0, hist_steps=1)
    s.set_launch(batched=True, graph_steps=every)
    t0 = time.perf_counter()
    n_eq = int(round(equil_tau / tau / every))
    for k in range(n_eq):
        s.step(every)
        if (k + 1) % max(1, n_eq // 4) == 0:
            _say(f"L={L} equilibration {k + 1}/{n_eq} x {every} steps, {time.perf_counter() - t0:.0f} s")
    n_s = int(round(prod_tau / tau / every))
    com = np.empty((n_s, n_boxes, 3))
    mids = np.empty((n_s, n_boxes, 2, 3))
    modes = np.empty((n_s, n_boxes, 5, 3))
    rg2 = np.empty((n_s, n_boxes))
    re2 = np.empty((n_s, n_boxes))
    kin = np.empty(n_s)
    snaps = []
    mid = [N // 2 - 1, N // 2]
    health = 0
    neg = 0.0          # populations n_i < 0 summed over samples and boxes (Sec. II.E)
    neg_max = 0.0      # the most in one box at one sample
    for k in range(n_s):
        s.step(every)
        obs = s.observables()
        for b, o in enumerate(obs):
            com[k, b], rg2[k, b], re2[k, b] = o["com"], o["rg2"], o["re2"]
            health |= o["health"]
            neg += o["neg"]
            neg_max = max(neg_max, o["neg"])
        x = s.bead_positions().reshape(n_boxes, N, 3)
        mids[k] = x[:, mid]
        modes[k] = an.rouse_modes(x, 5)
        if k % 20 == 0:
            snaps.append(x.copy())
        v = s.velocity_history(obs[0]["step"] - 1)
        kin[k] = float(np.mean(np.sum(v * v, axis=-1))) * base["mass"] / 3.0
        if (k + 1) % max(1, n_s // 10) == 0:
            _say(f"L={L} production {k + 1}/{n_s}, {time.perf_counter() - t0:.0f} s")
    wall = time.perf_counter() - t0
    s.close()

    # statics: per-box time averages, error from their spread across boxes
    def box_mean(a):
        m = a.mean(axis=0)
        return float(m.mean()), float(m.std(ddof=1) / np.sqrt(len(m)))

    res = {"L": L, "boxes": n_boxes, "precision": "fp32_dev" if prec == lbm.FP32_DEV else "fp64",
           "thermalize": "all modes" if therm == 2 else ("stress modes" if therm == 1 else "none"),
           "equil_tau": n_eq * every * tau, "prod_tau": n_s * every * tau, "sample_tau": every * tau,
           "lb_steps": (n_eq + n_s) * every, "wall_s": round(wall, 1), "health": int(health),
           # Sec. II.E chooses the LB step so that populations rarely go negative
           "negative_population_fraction": neg / (n_s * n_boxes * 19 * L ** 3),
           "negative_populations_max_per_box": int(neg_max)}
    res["re2"] = box_mean(re2)
    res["rg2"] = box_mean(rg2)
    ks = np.geomspace(0.3, 3.0, 24)
    sk = np.mean([an.structure_factor(c, ks) for c in snaps], axis=0)
    rh_box = np.mean([an.inverse_hydrodynamic_radius(c) for c in snaps], axis=0)   # per box
    res["inv_rh"] = (float(rh_box.mean()), float(rh_box.std(ddof=1) / np.sqrt(n_boxes)))
    res["nu"] = an.flory_exponent(ks, sk, 0.8, 2.0)
    lags = np.unique(np.round(np.geomspace(1, n_s // 4, 40)).astype(int))
    t = lags * every * tau
    g1 = an.msd(mids, lags)
    rel = mids - com[:, :, None, :]
    g2 = an.msd(rel, lags)
    g3_box = np.stack([an.msd(com[:, b], lags) for b in range(n_boxes)])
    g3 = g3_box.mean(axis=0)
    res["g1_exponent"] = an.power_law_exponent(t, g1, 20, 80)
    res["g3_exponent"] = an.power_law_exponent(t, g3, 20, 80)
    d_box = np.array([an.diffusion_constant(t, g, 20, 80) for g in g3_box])
    res["d_cm"] = (float(d_box.mean()), float(d_box.std(ddof=1) / np.sqrt(n_boxes)))
    d_long = np.array([an.diffusion_constant(t, g, 100, 1000) for g in g3_box])
    res["d_cm_100_1000"] = (float(d_long.mean()), float(d_long.std(ddof=1) / np.sqrt(n_boxes)))
    res["tau_tr"] = res["rg2"][0] / (6 * res["d_cm"][0])
    lag700 = np.array([int(round(700 / (every * tau)))])
    if lag700[0] < n_s:
        res["rouse1_acf_t700"] = float(an.autocorrelation(modes[:, :, 0], lag700)[0])
    res["kinetic_temperature_over_kT"] = float(kin.mean() / base["kT"])
    res["curves"] = {"t": t.tolist(), "g1": g1.tolist(), "g2": g2.tolist(), "g3": g3.tolist(),
                     "k": ks.tolist(), "S": sk.tolist()}
    if L in PAPER_TABLE1:
        res["paper"] = dict(PAPER_TABLE1[L])
        if therm == 1:
            res["paper"]["g1_exponent"] = PAPER_G1_STRESS_ONLY[L]
    return res


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--L", type=int, nargs="+", default=[10, 15, 25])
    ap.add_argument("--boxes", type=int, default=128)
    ap.add_argument("--equil-tau", type=float, default=2000.0)
    ap.add_argument("--prod-tau", type=float, default=10000.0)
    ap.add_argument("--sample-tau", type=float, default=1.0)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--therm", type=int, default=2, choices=[0, 1, 2],
                    help="thermalized modes: 2 all non-conserved, 1 stress only, 0 none")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    out = []
    for L in a.L:
        r = run_box_size(L, a.boxes, a.equil_tau, a.prod_tau, a.sample_tau, a.seed, therm=a.therm)
        brief = {k: v for k, v in r.items() if k != "curves"}
        _say(json.dumps(brief))
        out.append(r)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(out, f)
    return out


if __name__ == "__main__":
    main()
