"""MI355X (gfx950) fluctuating D3Q19 lattice Boltzmann with bead-spring coupling.

Python binding of ``liblbmd.so`` (C ABI in ``include/lbmd.h``): argument
marshalling only.  Every step of the method runs in the library's HIP
kernels; PyTorch provides device memory and the stream.  If the library is
not built this module raises on use: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbmd.so")

LB_OK, LB_EINVAL, LB_ENOMEM, LB_EDEVICE, LB_ENUMERIC, LB_ESTATE = 0, -1, -2, -3, -4, -5
FP64, FP32_DEV = 0, 1
N_COLLIDE_VARIANTS = 13
# launch shape of each collide variant (include/lbmd.h): nodes per workgroup,
# cap on waves per SIMD, grid form
COLLIDE_VARIANT_SHAPES = (
    [{"nodes_per_workgroup": 256, "max_waves_per_simd": w, "grid": "one workgroup per tile"} for w in range(4, 9)]
    + [{"nodes_per_workgroup": 256, "max_waves_per_simd": w, "grid": "n_CU x waves, strided"} for w in range(4, 9)]
    + [{"nodes_per_workgroup": 512, "max_waves_per_simd": 4, "grid": "one workgroup per tile"},
       {"nodes_per_workgroup": 512, "max_waves_per_simd": 6, "grid": "one workgroup per tile"},
       {"nodes_per_workgroup": 1024, "max_waves_per_simd": 4, "grid": "one workgroup per tile"}])
HEALTH = {"density": 0x1, "mach": 0x2, "fene": 0x4, "table": 0x8, "fixed": 0x10}


class LBError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"lbmd status {status}: {msg}")
        self.status = status


class BoxDesc(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int32), ("n_beads", ctypes.c_int32),
        ("rho0", ctypes.c_double), ("omega_shear", ctypes.c_double),
        ("omega_bulk", ctypes.c_double), ("omega_ghost", ctypes.c_double),
        ("kT", ctypes.c_double), ("thermalize", ctypes.c_int32),
        ("tau_lb", ctypes.c_double), ("md_dt", ctypes.c_double),
        ("md_substeps", ctypes.c_int32), ("bead_mass", ctypes.c_double),
        ("zeta", ctypes.c_double), ("k_fene", ctypes.c_double),
        ("r0_fene", ctypes.c_double), ("eps_wca", ctypes.c_double),
        ("sigma_wca", ctypes.c_double), ("seed", ctypes.c_uint32),
        ("box_id", ctypes.c_uint32), ("chain_len", ctypes.c_int32),
    ]


class Obs(ctypes.Structure):
    _fields_ = [
        ("mass", ctypes.c_double), ("j_lat", ctypes.c_double * 3),
        ("p_fluid", ctypes.c_double * 3), ("p_beads", ctypes.c_double * 3),
        ("p_total", ctypes.c_double * 3), ("com", ctypes.c_double * 3),
        ("rg2", ctypes.c_double), ("re2", ctypes.c_double),
        ("neg_count", ctypes.c_double), ("mode_sq", ctypes.c_double * 19),
        ("health", ctypes.c_uint32), ("nlist_builds", ctypes.c_uint32), ("step", ctypes.c_uint64),
    ]


_lib = None


def lib() -> ctypes.CDLL:
    """Load liblbmd.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run paper_0903_5067_amd/build.py "
                               "(or __graft_entry__.build()) first; there is no fallback")
        L = ctypes.CDLL(LIB_PATH)
        vp, sz, i32, i64 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int64
        bdp = ctypes.POINTER(BoxDesc)
        L.lb_query_sizes.argtypes = [bdp, i32, i32, i32, ctypes.POINTER(sz), ctypes.POINTER(sz)]
        L.lb_init.argtypes = [bdp, i32, i32, i32, ctypes.POINTER(ctypes.c_double), vp, vp, vp,
                              ctypes.POINTER(vp)]
        L.lb_couple.argtypes = [vp]
        L.lb_step.argtypes = [vp, i64]
        L.lb_observables.argtypes = [vp, ctypes.POINTER(Obs)]
        L.lb_observables_static.argtypes = [vp, ctypes.POINTER(Obs)]
        L.lb_state_host_bytes.argtypes = [vp]
        L.lb_state_host_bytes.restype = sz
        L.lb_export_state.argtypes = [vp, vp, sz]
        L.lb_import_state.argtypes = [vp, vp, sz]
        L.lb_pending_impulse.argtypes = [vp, ctypes.POINTER(ctypes.c_double), sz]
        L.lb_velocity_history.argtypes = [vp, i64, ctypes.POINTER(ctypes.c_double), sz]
        L.lb_bead_positions.argtypes = [vp, ctypes.POINTER(ctypes.c_double), sz]
        L.lb_set_launch.argtypes = [vp, i32, i32]
        L.lb_collide_only.argtypes = [vp, i32]
        L.lb_autotune.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(i32)]
        L.lb_set_collide_variant.argtypes = [vp, i32]
        L.lb_stream.argtypes = [vp]
        L.lb_stream.restype = vp
        L.lb_window_bytes.argtypes = [vp, i32, i32]
        L.lb_window_bytes.restype = sz
        L.lb_window_forward.argtypes = [vp, vp, sz, i32, i32, ctypes.POINTER(ctypes.c_double)]
        L.lb_window_backward.argtypes = [vp, vp, sz, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        L.lb_window_rewind.argtypes = [vp, vp, sz]
        L.lb_set_rates.argtypes = [vp, i32, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.lb_free.argtypes = [vp]
        L.lb_free.restype = None
        L.lb_last_error.argtypes = [vp]
        L.lb_last_error.restype = ctypes.c_char_p
        for name in ("lb_query_sizes", "lb_init", "lb_couple", "lb_step", "lb_observables", "lb_observables_static",
                     "lb_export_state", "lb_import_state", "lb_pending_impulse",
                     "lb_velocity_history", "lb_bead_positions", "lb_set_launch", "lb_collide_only", "lb_window_forward",
                     "lb_window_backward", "lb_window_rewind", "lb_set_rates", "lb_autotune",
                     "lb_set_collide_variant"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(st: int, handle=None):
    if st != LB_OK:
        msg = lib().lb_last_error(handle).decode()
        raise LBError(st, msg)


def make_desc(p: dict) -> BoxDesc:
    d = BoxDesc()
    d.L, d.n_beads = int(p["L"]), int(p["N"])
    d.rho0, d.omega_shear, d.omega_bulk, d.omega_ghost = p["rho0"], p["omega_s"], p["omega_b"], p["omega_g"]
    d.kT, d.thermalize = p["kT"], int(p["therm"])
    d.tau_lb, d.md_dt, d.md_substeps = p["tau_lb"], p["md_dt"], int(p["md_substeps"])
    d.bead_mass, d.zeta, d.k_fene, d.r0_fene = p["mass"], p["zeta"], p["k_fene"], p["r0_fene"]
    d.eps_wca, d.sigma_wca = p["eps_wca"], p["sigma_wca"]
    d.seed, d.box_id = int(p["seed"]), int(p["box_id"])
    d.chain_len = int(p.get("chain_len", 0))
    return d


def query_sizes(boxes: list[dict], precision: int, hist_steps: int = 0):
    arr = (BoxDesc * len(boxes))(*[make_desc(b) for b in boxes])
    s, c = ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib().lb_query_sizes(arr, len(boxes), precision, hist_steps, ctypes.byref(s), ctypes.byref(c)))
    return s.value, c.value


class LBSystem:
    """A batch of independent boxes living in device memory.

    boxes: list of parameter dicts (keys as in ``lbinputs.BOX_FIELDS``);
    bead_x0: float64 array [sum N, 3] (host) of initial bead positions.
    """

    def __init__(self, boxes: list[dict], precision: int = FP32_DEV, bead_x0=None,
                 hist_steps: int = 0, device: str = "cuda:0"):
        import torch
        self.boxes = [dict(b) for b in boxes]
        self.precision = precision
        self.hist_steps = hist_steps
        self.device = torch.device(device)
        arr = (BoxDesc * len(boxes))(*[make_desc(b) for b in boxes])
        self._arr = arr
        sb, cb = query_sizes(boxes, precision, hist_steps)
        self.state = torch.empty(max(sb, 256), dtype=torch.uint8, device=self.device)
        self.scratch = torch.empty(max(cb, 256), dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.Stream(device=self.device)
        n_beads = sum(int(b["N"]) for b in boxes)
        x0p = None
        if n_beads:
            x0 = np.ascontiguousarray(bead_x0, dtype=np.float64).reshape(n_beads, 3)
            self._x0 = x0
            x0p = x0.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        h = ctypes.c_void_p()
        _check(lib().lb_init(arr, len(boxes), precision, hist_steps, x0p,
                             ctypes.c_void_p(self.state.data_ptr()), ctypes.c_void_p(self.scratch.data_ptr()),
                             ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self.h = h
        self.n_beads = n_beads

    # -- the path ---------------------------------------------------------
    def couple(self):
        _check(lib().lb_couple(self.h), self.h)

    def step(self, n: int = 1):
        _check(lib().lb_step(self.h, int(n)), self.h)

    def set_launch(self, batched: bool = True, graph_steps: int = 0, overlap: bool = True,
                   resident: bool = True):
        """Launch structure of step (lb_set_launch): batched or per box,
        graph_steps per HIP graph (0: direct launches), overlap False to
        re-collide the chain's nodes after the collide, resident False to keep
        every chain kernel from waiting for a later collide (for tools that
        run one kernel at a time)."""
        mode = ((3 if not resident else 1) if overlap else 2) if batched else 0
        _check(lib().lb_set_launch(self.h, mode, int(graph_steps)), self.h)

    def collide_only(self, n: int = 1):
        """n launches of the fused collide+stream kernel, state not advanced."""
        _check(lib().lb_collide_only(self.h, int(n)), self.h)

    def autotune(self, reps: int = 20):
        """Time every launch shape of the collide+stream kernel on this state
        and keep the fastest; returns (chosen variant, microseconds per launch
        of each variant)."""
        t = (ctypes.c_float * N_COLLIDE_VARIANTS)()
        ch = ctypes.c_int32()
        _check(lib().lb_autotune(self.h, int(reps), t, ctypes.byref(ch)), self.h)
        return ch.value, [float(v) for v in t]

    def set_collide_variant(self, variant: int):
        _check(lib().lb_set_collide_variant(self.h, int(variant)), self.h)

    def synchronize(self):
        self.stream.synchronize()

    # -- observation ------------------------------------------------------
    def observables(self, allow_unhealthy: bool = False, static: bool = False) -> list[dict]:
        """Observables of every box (lb_observables); static=True takes the
        entry point that allocates nothing (lb_observables_static)."""
        out = (Obs * len(self.boxes))()
        st = (lib().lb_observables_static if static else lib().lb_observables)(self.h, out)
        if st != LB_OK and not (allow_unhealthy and st == LB_ENUMERIC):
            _check(st, self.h)
        res = []
        for o in out:
            res.append({"mass": o.mass, "j_lat": np.array(o.j_lat), "p_fluid": np.array(o.p_fluid),
                        "p_beads": np.array(o.p_beads), "p_total": np.array(o.p_total),
                        "com": np.array(o.com), "rg2": o.rg2, "re2": o.re2, "neg": o.neg_count,
                        "mode_sq": np.array(o.mode_sq), "health": o.health, "step": o.step,
                        "nlist_builds": o.nlist_builds})
        return res

    def export_state(self) -> dict:
        nbytes = lib().lb_state_host_bytes(self.h)
        buf = np.zeros(nbytes // 8, dtype=np.float64)
        _check(lib().lb_export_state(self.h, buf.ctypes.data_as(ctypes.c_void_p), nbytes), self.h)
        return self._split(buf)

    def import_state(self, state: dict):
        buf = self._join(state)
        _check(lib().lb_import_state(self.h, buf.ctypes.data_as(ctypes.c_void_p), buf.nbytes), self.h)

    def _split(self, buf: np.ndarray) -> dict:
        step = int(buf[:1].view(np.uint64)[0])
        o = 1
        boxes = []
        for b in self.boxes:
            L, N = int(b["L"]), int(b["N"])
            V = L ** 3
            n = buf[o:o + 19 * V].reshape(19, L, L, L).copy()
            o += 19 * V
            arrs = []
            for _ in range(4):
                arrs.append(buf[o:o + 3 * N].reshape(N, 3).copy())
                o += 3 * N
            boxes.append({"n": n, "x": arrs[0], "v": arrs[1], "f": arrs[2], "fc": arrs[3]})
        return {"step": step, "boxes": boxes}

    def _join(self, state: dict) -> np.ndarray:
        parts = [np.array([state["step"]], dtype=np.uint64).view(np.float64)]
        for b, s in zip(self.boxes, state["boxes"]):
            parts.append(np.ascontiguousarray(s["n"], dtype=np.float64).reshape(-1))
            for k in ("x", "v", "f", "fc"):
                parts.append(np.ascontiguousarray(s[k], dtype=np.float64).reshape(-1))
        return np.ascontiguousarray(np.concatenate(parts))

    def pending_impulse(self) -> list[np.ndarray]:
        total = sum(3 * int(b["L"]) ** 3 for b in self.boxes)
        buf = np.zeros(total)
        _check(lib().lb_pending_impulse(self.h, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                        buf.nbytes), self.h)
        out, o = [], 0
        for b in self.boxes:
            L = int(b["L"])
            out.append(buf[o:o + 3 * L ** 3].reshape(3, L, L, L))
            o += 3 * L ** 3
        return out

    def velocity_history(self, step: int) -> np.ndarray:
        buf = np.zeros((max(self.n_beads, 1), 3))
        _check(lib().lb_velocity_history(self.h, int(step), buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                         buf.nbytes), self.h)
        return buf[: self.n_beads]

    def bead_positions(self) -> np.ndarray:
        """Unwrapped bead positions [sum N, 3] at the current step boundary."""
        buf = np.zeros((max(self.n_beads, 1), 3))
        _check(lib().lb_bead_positions(self.h, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), buf.nbytes),
               self.h)
        return buf[: self.n_beads]

    # -- adjoint window ---------------------------------------------------
    def set_rates(self, box: int, omega_shear: float, omega_bulk: float, zeta: float):
        _check(lib().lb_set_rates(self.h, int(box), float(omega_shear), float(omega_bulk), float(zeta)), self.h)
        b = self.boxes[box]
        b["omega_s"], b["omega_b"], b["zeta"] = float(omega_shear), float(omega_bulk), float(zeta)

    def window_forward(self, T: int, k: int) -> np.ndarray:
        """T steps with checkpoints every k; bead velocities after each step [T, sum N, 3]."""
        import torch
        need = lib().lb_window_bytes(self.h, int(T), int(k))
        if getattr(self, "_ws", None) is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        vh = np.zeros((T, max(self.n_beads, 1), 3))
        _check(lib().lb_window_forward(self.h, ctypes.c_void_p(self._ws.data_ptr()), self._ws.numel(), int(T), int(k),
                                       vh.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), self.h)
        return vh[:, : self.n_beads]

    def window_backward(self, dj_dv: np.ndarray) -> np.ndarray:
        """dJ/dv [T, sum N, 3] -> dJ/d(omega_shear, omega_bulk, zeta) per box [n_boxes, 3]."""
        dj = np.ascontiguousarray(dj_dv, dtype=np.float64)
        grad = np.zeros((len(self.boxes), 3))
        _check(lib().lb_window_backward(self.h, ctypes.c_void_p(self._ws.data_ptr()), self._ws.numel(),
                                        dj.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                        grad.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), self.h)
        return grad

    def window_rewind(self):
        _check(lib().lb_window_rewind(self.h, ctypes.c_void_p(self._ws.data_ptr()), self._ws.numel()), self.h)

    def close(self):
        if getattr(self, "h", None):
            lib().lb_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
