"""Helpers shared by the GPU parity tests: run the same seeded case through the
HIP library (via the C ABI binding) and through the oracle."""
from __future__ import annotations

import sys

import numpy as np

import lbinputs


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def params(preset="plain16", **kw):
    return lbinputs.box_params(preset, **kw)


def initial_pops(orc, p, amp=0.0, seed=0):
    """Full populations w_i rho0 (1 + amp * U(-1,1)) as a (19, L, L, L) array."""
    c, w, e, b = orc.tables()
    L = int(p["L"])
    n = w[:, None, None, None] * p["rho0"] * np.ones((19, L, L, L))
    if amp:
        n = n * (1.0 + lbinputs.random_deviations(L, amp, seed))
    return n


def chain(p, seed=None):
    """Initial beads of box p: one chain, or N / chain_len chains."""
    return lbinputs.initial_chains(p, seed)


def gpu_system(boxes, precision, xs=None, pops=None, hist_steps=0):
    """LBSystem over `boxes` with initial bead positions xs (list per box) and
    optional initial populations (list per box, None = rest state)."""
    import paper_0903_5067_amd as lbm
    x0 = None
    if any(int(b["N"]) for b in boxes):
        x0 = np.concatenate([x for x in xs if len(x)], axis=0)
    sys_ = lbm.LBSystem(boxes, precision=precision, bead_x0=x0, hist_steps=hist_steps)
    if pops is not None:
        st = sys_.export_state()
        for bst, n in zip(st["boxes"], pops):
            if n is not None:
                bst["n"][...] = n
        sys_.import_state(st)
    return sys_


def oracle_state(orc, p, n, x=None):
    bx = orc.make_box(**p)
    return orc.State(bx, n, x if int(p["N"]) else None)


def max_rel_pop_err(n_gpu, n_orc, orc, rho0=1.0):
    c, w, e, b = orc.tables()
    return float(np.max(np.abs(n_gpu - n_orc) / (w[:, None, None, None] * rho0)))
