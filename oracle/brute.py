"""Brute-force numpy statement of one LB collide+stream step, for tiny lattices.

TEST INFRASTRUCTURE ONLY.  Independent of ``lbmd_oracle.c``: it builds the
19x19 mode matrix from the polynomial definitions, inverts it with a dense
solver instead of using the weighted-transpose formula, takes the equilibrium
in population space from the second-order expansion of Sec. II.B and projects
it, takes the forcing as the population-space second-order (Guo-type) source
projected onto the modes, relaxes every mode with the same formula, and moves
populations with an explicit permutation.  Its Philox4x32-10 is a separate
numpy implementation of the published generator.
"""
from __future__ import annotations

import itertools

import numpy as np

M0, M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = np.uint64(0xFFFFFFFF)


def philox(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10 on uint64 arrays holding 32-bit values."""
    c = [np.asarray(v, dtype=np.uint64) & MASK for v in (c0, c1, c2, c3)]
    k0 = np.uint64(k0 & 0xFFFFFFFF)
    k1 = np.uint64(k1 & 0xFFFFFFFF)
    for rnd in range(10):
        if rnd:
            k0 = np.uint64((int(k0) + W0) & 0xFFFFFFFF)
            k1 = np.uint64((int(k1) + W1) & 0xFFFFFFFF)
        p0 = M0 * c[0]
        p1 = M1 * c[2]
        c = [((p1 >> np.uint64(32)) ^ c[1] ^ k0) & MASK, p1 & MASK,
             ((p0 >> np.uint64(32)) ^ c[3] ^ k1) & MASK, p0 & MASK]
    return c


def velocities():
    """D3Q19: rest, the 6 face and the 12 edge neighbours, in the library order."""
    c = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
    for a, b in ((0, 1), (0, 2), (1, 2)):
        for sa, sb in ((1, 1), (1, -1), (-1, 1), (-1, -1)):
            v = [0, 0, 0]
            v[a], v[b] = sa, sb
            c.append(tuple(v))
    c = np.array(c, dtype=np.float64)
    w = np.array([{0: 1 / 3, 1: 1 / 18, 2: 1 / 36}[int(round(s))] for s in (c * c).sum(1)])
    return c, w


def mode_matrix(c):
    cx, cy, cz = c[:, 0], c[:, 1], c[:, 2]
    c2 = cx ** 2 + cy ** 2 + cz ** 2
    rows = [np.ones_like(cx), cx, cy, cz, c2 - 1, 3 * cx ** 2 - c2, cy ** 2 - cz ** 2,
            cx * cy, cy * cz, cx * cz, (3 * c2 - 5) * cx, (3 * c2 - 5) * cy, (3 * c2 - 5) * cz,
            (cy ** 2 - cz ** 2) * cx, (cz ** 2 - cx ** 2) * cy, (cx ** 2 - cy ** 2) * cz,
            3 * c2 ** 2 - 6 * c2 + 1, (2 * c2 - 3) * (3 * cx ** 2 - c2),
            (2 * c2 - 3) * (cy ** 2 - cz ** 2)]
    return np.array(rows)


def step(n, dp, p, t):
    """One collide+stream step.  n: (19, L, L, L) full populations, dp: (3, L, L, L)
    lattice-unit impulse, p: parameter dict, t: step index."""
    c, w = velocities()
    M = mode_matrix(c)
    Minv = np.linalg.inv(M)
    b = (M ** 2 * w).sum(1)
    L = n.shape[1]
    cs2 = 1.0 / 3.0
    nn = n.reshape(19, -1)
    f = dp.reshape(3, -1)
    m = M @ nn
    rho = nn.sum(0)
    j = c.T @ nn
    u = (j + 0.5 * f) / rho
    cu = c @ u                                   # (19, V)
    usq = (u * u).sum(0)
    neq = w[:, None] * rho * (1 + cu / cs2 + cu ** 2 / (2 * cs2 ** 2) - usq / (2 * cs2))
    cf = c @ f
    uf = (u * f).sum(0)
    # population-space second-order source for an impulse f per step
    src = w[:, None] * ((cf - uf) / cs2 + cu * cf / cs2 ** 2)
    meq = M @ neq
    S = M @ src
    gam = np.zeros(19)
    gam[4] = 1 - p["omega_b"]
    gam[5:10] = 1 - p["omega_s"]
    gam[10:] = 1 - p["omega_g"]
    ms = meq + gam[:, None] * (m - meq) + 0.5 * (1 + gam)[:, None] * S
    kT_lat = p["kT"] * p["tau_lb"] ** 2
    mu = kT_lat / cs2
    last = {2: 18, 1: 9, 0: 3}[p["therm"]]
    V = nn.shape[1]
    node = np.arange(V, dtype=np.uint64)
    words = []
    for blk in range(4):
        words += philox(node, t, 0, blk, p["seed"], p["box_id"])
    for k in range(4, last + 1):
        wd = words[k - 4].astype(np.int64) >> 8
        r = np.sqrt(12.0) * ((2 * wd - (1 << 24) + 1) * 2.0 ** -25)
        ms[k] += np.sqrt(mu * rho * b[k] * (1 - gam[k] ** 2)) * r
    ns = (Minv @ ms).reshape(19, L, L, L)
    out = np.empty_like(ns)
    for i in range(19):
        # n_i(r + c_i) = n*_i(r); axes of the array are (z, y, x)
        out[i] = np.roll(ns[i], shift=(int(c[i, 2]), int(c[i, 1]), int(c[i, 0])), axis=(0, 1, 2))
    return out


def equilibrium(rho, u):
    """Second-order equilibrium of Sec. II.B for arrays rho (V,), u (3, V)."""
    c, w = velocities()
    cs2 = 1.0 / 3.0
    cu = c @ u
    usq = (u * u).sum(0)
    return w[:, None] * rho * (1 + cu / cs2 + cu ** 2 / (2 * cs2 ** 2) - usq / (2 * cs2))


def all_permutation_check(L):
    """Each population moves to exactly one node: the streaming is a permutation."""
    c, _ = velocities()
    for i in range(19):
        seen = set()
        for x, y, z in itertools.product(range(L), repeat=3):
            seen.add(((x + int(c[i, 0])) % L, (y + int(c[i, 1])) % L, (z + int(c[i, 2])) % L))
        assert len(seen) == L ** 3
