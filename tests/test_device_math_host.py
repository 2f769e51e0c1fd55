"""The device collision (lbmd_device.hpp) compiled for the host and compared
with the oracle node by node: catches arithmetic mistakes in the kernel's
mode transform, relaxation and noise before any GPU run."""
from __future__ import annotations

import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

import lbinputs

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def host_lib(tmp_path_factory):
    if shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    out = tmp_path_factory.mktemp("hc") / "host_collide.so"
    subprocess.run(["hipcc", "-O2", "-fPIC", "-shared", "-o", str(out),
                    os.path.join(HERE, "native", "host_collide.cpp")], check=True, capture_output=True)
    lib = ctypes.CDLL(str(out))
    dp = ctypes.POINTER(ctypes.c_double)
    for f in (lib.host_collide_f64, lib.host_collide_f32):
        f.argtypes = [dp, dp] + [ctypes.c_double] * 6 + [ctypes.c_int] + [ctypes.c_uint] * 4 + [dp]
    return lib


@pytest.mark.parametrize("therm", [0, 1, 2])
def test_host_build_of_device_collision_matches_oracle(orc, host_lib, therm):
    c, w, e, b = orc.tables()
    rng = np.random.default_rng(therm)
    dpp = ctypes.POINTER(ctypes.c_double)
    for _ in range(40):
        ws, wb, wg = rng.uniform(0.3, 1.9, 3)
        kT, tau = 0.3, 0.1
        n = w * (1 + rng.uniform(-0.2, 0.2, 19))
        dp = rng.uniform(-0.01, 0.01, 3)
        node, step = int(rng.integers(0, 2 ** 30)), int(rng.integers(0, 2 ** 20))
        p = lbinputs.box_params("plain16", L=4, N=0, kT=kT, omega_s=ws, omega_b=wb, omega_g=wg,
                                therm=therm, seed=77, box_id=3)
        ref = orc.collide_one(orc.make_box(**p), n, dp, node, step)
        for f, tol in ((host_lib.host_collide_f64, 1e-14), (host_lib.host_collide_f32, 5e-7)):
            out = np.zeros(19)
            f(n.ctypes.data_as(dpp), dp.ctypes.data_as(dpp), 1.0, ws, wb, wg, kT, tau, therm, node, step,
              77, 3, out.ctypes.data_as(dpp))
            assert np.max(np.abs(out - ref) / w) < tol
