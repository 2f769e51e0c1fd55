"""CPU checks of the C ABI: the library loads, exports every function the
header declares, sizes buffers and rejects invalid problems before touching a
device (no GPU needed)."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

import lbinputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lbm():
    import paper_0903_5067_amd as m
    if not os.path.exists(m.LIB_PATH):
        pytest.skip("liblbmd.so not built")
    m.lib()
    return m


def test_exports_every_declared_symbol(lbm):
    hdr = open(os.path.join(ROOT, "include", "lbmd.h")).read()
    names = sorted(set(re.findall(r"\b(lb_[a-z_]+)\s*\(", hdr)))
    assert len(names) >= 12
    L = lbm.lib()
    for n in names:
        assert hasattr(L, n), n


def test_binding_refuses_missing_library(monkeypatch, tmp_path):
    import paper_0903_5067_amd as m
    monkeypatch.setattr(m, "_lib", None)
    monkeypatch.setattr(m, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(RuntimeError):
        m.lib()


def _sizes(lbm, boxes, prec=1, hist=0):
    return lbm.query_sizes(boxes, prec, hist)


def test_query_sizes_layout(lbm):
    p = lbinputs.box_params("prec256")
    s32, c32 = _sizes(lbm, [p], 1)
    s64, c64 = _sizes(lbm, [p], 0)
    V = 256 ** 3
    # two FP32 deviation buffers of 19 planes plus FP64 bead arrays
    assert 2 * 19 * V * 4 <= s32 < 2 * 19 * V * 4 * 1.01
    assert 2 * 19 * V * 8 <= s64 < 2 * 19 * V * 8 * 1.01
    # scratch: dense fixed-point node impulses (24 B), fix-up stamps (4 B) and,
    # with a chain above 256 beads, overflow marks (4 B) per node
    assert 32 * V <= c32 < 32 * V + 64 * 2 ** 20
    b = [lbinputs.box_params("plain16", L=L, N=N) for L, N in lbinputs.batched_table(256, 1)]
    sb, cb = _sizes(lbm, b, 1)
    nodes = sum(L ** 3 for L, _ in lbinputs.batched_table(256, 1))
    assert sb >= 2 * 19 * nodes * 4


@pytest.mark.parametrize("bad", [dict(L=1), dict(omega_s=2.0), dict(omega_b=0.0), dict(kT=-1.0),
                                 dict(md_substeps=5), dict(therm=3), dict(N=2000), dict(rho0=0.0),
                                 dict(L=4, N=65), dict(N=10, chain_len=3), dict(chain_len=-1)])
def test_invalid_parameters_rejected(lbm, bad):
    p = lbinputs.box_params("plain16", **bad)
    with pytest.raises(lbm.LBError) as ei:
        _sizes(lbm, [p])
    assert ei.value.status == lbm.LB_EINVAL


def test_overstretched_initial_bond_rejected_before_device_work(lbm):
    p = lbinputs.box_params("plain16", L=8, N=3)
    arr = (lbm.BoxDesc * 1)(lbm.make_desc(p))
    x = (ctypes.c_double * 9)(1, 1, 1, 2, 1, 1, 3.6, 1, 1)    # second bond 1.6 > R0 = 1.5
    h = ctypes.c_void_p()
    st = lbm.lib().lb_init(arr, 1, 1, 0, x, ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 21), None,
                           ctypes.byref(h))
    assert st == lbm.LB_EINVAL
    assert b"R0" in lbm.lib().lb_last_error(None)


def test_overstretched_bond_inside_a_chain_rejected(lbm):
    """With two chains of three beads the gap between bead 2 and bead 3 is no
    bond; a stretched bond inside the second chain still is."""
    p = lbinputs.box_params("plain16", L=8, N=6, chain_len=3)
    arr = (lbm.BoxDesc * 1)(lbm.make_desc(p))
    x = (ctypes.c_double * 18)(1, 1, 1, 2, 1, 1, 3, 1, 1, 5, 5, 5, 6, 5, 5, 7.6, 5, 5)
    h = ctypes.c_void_p()
    st = lbm.lib().lb_init(arr, 1, 1, 0, x, ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 21), None,
                           ctypes.byref(h))
    assert st == lbm.LB_EINVAL
    assert b"R0" in lbm.lib().lb_last_error(None)


def test_unaligned_buffers_rejected(lbm):
    p = lbinputs.box_params("plain16", L=8, N=0)
    arr = (lbm.BoxDesc * 1)(lbm.make_desc(p))
    h = ctypes.c_void_p()
    st = lbm.lib().lb_init(arr, 1, 1, 0, None, ctypes.c_void_p((1 << 20) + 4), ctypes.c_void_p(1 << 21),
                           None, ctypes.byref(h))
    assert st == lbm.LB_EINVAL
