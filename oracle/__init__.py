"""FP64 CPU oracle for the fluctuating D3Q19 LB step with bead coupling.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  Nothing in the GPU library imports
or links this package, and this package imports nothing from the GPU library.

The arithmetic lives in ``lbmd_oracle.cpp`` (plain C++, FP64, no code shared
with the HIP path; written once over the scalar type so that a dual-number
instantiation gives exact forward-mode derivatives with respect to the shear
and bulk rates and the friction); this module builds it and marshals arrays.
``brute.py`` is a second, independent numpy statement of one collide+stream
step on tiny lattices, used to pin the C oracle.

Parity status per function (what pins it is listed in the test files):
  philox4x32_10        pinned (published known-answer vectors, rocRAND source)
  tables               pinned (exact weight/moment identities, orthogonality)
  collide_stream       pinned (brute force, equilibrium, conservation,
                               equipartition, shear and sound damping)
  couple               pinned (force = -grad V, exact linear interpolation,
                               momentum invariant, bead equipartition; the
                               substep order: a free chain's energy has no
                               drift and second-order fluctuation, which
                               planted reorderings fail; several chains per
                               box: -grad V with bonds along each chain only,
                               far-apart chains move bit for bit as they do
                               alone)
  observables          pinned (closed forms on hand-made states, one chain
                               and several rods; negative-population count on
                               states with a known count)
  window_tangent       pinned (central finite differences of the oracle's own
                               window; values identical to run())
  specific noise realisations / long trajectories: parity unpinned beyond the
  shared generator (any realisation with the right moments is valid).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbmd_oracle.cpp")
_LIB = os.path.join(_HERE, "liblbmd_oracle.so")

OBS_LEN = 38
OBS = {
    "mass": 0, "j_lat": slice(1, 4), "p_fluid": slice(4, 7), "p_beads": slice(7, 10),
    "p_total": slice(10, 13), "com": slice(13, 16), "rg2": 16, "re2": 17,
    "neg": 18, "mode_sq": slice(19, 38),
}


TUNED_FLAGS = ["-O3", "-march=native"]


def build(verbose: bool = False, out: str | None = None, tuned: bool = False) -> str:
    """Compile the oracle with g++: plain -O2 (the portable build the tests
    load), or with ``tuned`` -O3 -march=native for the host it is built on
    (the timed CPU baseline; built where it runs, since the instruction set
    differs between hosts).  Never fast-math, never FMA contraction, so both
    builds compute the same bits."""
    dst = out or _LIB
    opt = TUNED_FLAGS if tuned else ["-O2"]
    cmd = ["g++", *opt, "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
           "-o", dst + ".tmp", _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(dst + ".tmp", dst)
    return dst


class Box(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int32), ("N", ctypes.c_int32),
        ("rho0", ctypes.c_double), ("omega_s", ctypes.c_double),
        ("omega_b", ctypes.c_double), ("omega_g", ctypes.c_double),
        ("kT", ctypes.c_double), ("therm", ctypes.c_int32),
        ("tau_lb", ctypes.c_double), ("md_dt", ctypes.c_double),
        ("md_substeps", ctypes.c_int32),
        ("mass", ctypes.c_double), ("zeta", ctypes.c_double),
        ("k_fene", ctypes.c_double), ("r0_fene", ctypes.c_double),
        ("eps_wca", ctypes.c_double), ("sigma_wca", ctypes.c_double),
        ("seed", ctypes.c_uint32), ("box_id", ctypes.c_uint32),
        ("chain_len", ctypes.c_int32),
    ]


_lib = None


def use_tuned_build(directory: str) -> str:
    """Build the -O3 -march=native oracle into ``directory`` and route every
    later call of this module to it (for timing on the host that runs it).
    Returns the library path."""
    global _lib
    path = build(out=os.path.join(directory, "liblbmd_oracle_tuned.so"), tuned=True)
    _lib = None
    lib(path)
    return path


def lib(path: str | None = None):
    global _lib
    if _lib is None:
        if path is None:
            path = _LIB
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
        _lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        bp = ctypes.POINTER(Box)
        _lib.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        _lib.orc_tables.argtypes = [dp, dp, dp, dp]
        _lib.orc_unit_noise.argtypes = [ctypes.c_uint32]
        _lib.orc_unit_noise.restype = ctypes.c_double
        _lib.orc_collide_stream.argtypes = [bp, dp, dp, dp, ctypes.c_uint32]
        _lib.orc_collide_one.argtypes = [bp, dp, dp, ctypes.c_uint32, ctypes.c_uint32, dp]
        _lib.orc_initial_forces.argtypes = [bp, dp, dp]
        _lib.orc_couple.argtypes = [bp, dp, dp, dp, dp, dp, ctypes.c_uint32, dp]
        _lib.orc_run.argtypes = [bp, dp, dp, dp, dp, dp, ctypes.c_uint32, ctypes.c_int32, dp]
        _lib.orc_observables.argtypes = [bp, dp, dp, dp, dp, dp]
        _lib.orc_window_tangent.argtypes = [bp, dp, dp, dp, dp, dp, ctypes.c_uint32, ctypes.c_int32, dp, dp]
        _lib.orc_num_threads.restype = ctypes.c_int
        _lib.orc_set_threads.argtypes = [ctypes.c_int]
    return _lib


def _p(a: np.ndarray | None):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_box(**kw) -> Box:
    b = Box()
    for name, _ in Box._fields_:
        setattr(b, name, kw.get(name, 0) if name == "chain_len" else kw[name])
    return b


def philox4x32_10(ctr, key) -> np.ndarray:
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def unit_noise(word: int) -> float:
    return lib().orc_unit_noise(int(word) & 0xFFFFFFFF)


def tables():
    c = np.zeros((19, 3)); w = np.zeros(19); e = np.zeros((19, 19)); b = np.zeros(19)
    lib().orc_tables(_p(c), _p(w), _p(e), _p(b))
    return c, w, e, b


class State:
    """Oracle state: populations n[19, L, L, L] (z, y, x order) plus chain."""

    def __init__(self, box: Box, n: np.ndarray, x: np.ndarray | None = None):
        self.box = box
        L, N = box.L, box.N
        self.n = np.ascontiguousarray(n, dtype=np.float64).reshape(19, L, L, L).copy()
        self.x = np.zeros((max(N, 1), 3)) if x is None else np.ascontiguousarray(x, dtype=np.float64).copy()
        self.v = np.zeros_like(self.x)
        self.f = np.zeros_like(self.x)
        self.fc = np.zeros_like(self.x)
        if N > 0:
            lib().orc_initial_forces(ctypes.byref(box), _p(self.x), _p(self.f))
        self.t = 0

    def copy(self) -> "State":
        s = State.__new__(State)
        s.box = self.box
        s.n, s.x, s.v, s.f, s.fc = (a.copy() for a in (self.n, self.x, self.v, self.f, self.fc))
        s.t = self.t
        return s

    def run(self, n_steps: int, record_velocities: bool = False):
        hist = np.zeros((n_steps, max(self.box.N, 1), 3)) if record_velocities else None
        lib().orc_run(ctypes.byref(self.box), _p(self.n), _p(self.x), _p(self.v), _p(self.f),
                      _p(self.fc), self.t, n_steps, _p(hist))
        self.t += n_steps
        return hist

    def window_tangent(self, n_steps: int):
        """Advance n_steps like run(); return the bead velocities at the end of
        each step [T, N, 3] and their derivatives with respect to
        (omega_shear, omega_bulk, zeta) [T, N, 3, 3] (forward mode, exact)."""
        N = self.box.N
        hist = np.zeros((n_steps, N, 3))
        dh = np.zeros((n_steps, N, 3, 3))
        lib().orc_window_tangent(ctypes.byref(self.box), _p(self.n), _p(self.x), _p(self.v), _p(self.f),
                                 _p(self.fc), self.t, n_steps, _p(hist), _p(dh))
        self.t += n_steps
        return hist, dh

    def couple(self) -> np.ndarray:
        L = self.box.L
        dp = np.zeros((3, L, L, L))
        lib().orc_couple(ctypes.byref(self.box), _p(self.n), _p(self.x), _p(self.v), _p(self.f),
                         _p(self.fc), self.t, _p(dp))
        return dp

    def collide_stream(self, dp: np.ndarray | None = None):
        out = np.empty_like(self.n)
        lib().orc_collide_stream(ctypes.byref(self.box), _p(self.n), _p(out),
                                 _p(None if dp is None else np.ascontiguousarray(dp)), self.t)
        self.n = out
        self.t += 1

    def observables(self) -> np.ndarray:
        out = np.zeros(OBS_LEN)
        lib().orc_observables(ctypes.byref(self.box), _p(self.n), _p(self.x), _p(self.v),
                              _p(self.fc), _p(out))
        return out


def collide_one(box: Box, n19, dp3=None, r: int = 0, t: int = 0) -> np.ndarray:
    n = np.ascontiguousarray(n19, dtype=np.float64)
    out = np.zeros(19)
    d = None if dp3 is None else np.ascontiguousarray(dp3, dtype=np.float64)
    lib().orc_collide_one(ctypes.byref(box), _p(n), _p(d), r, t, _p(out))
    return out


def initial_forces(box: Box, x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    f = np.zeros_like(x)
    lib().orc_initial_forces(ctypes.byref(box), _p(x), _p(f))
    return f


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))
