"""Throughput of the fluctuating D3Q19 LB step with bead coupling on one MI355X.

One step = one full LB step through every stage of the path: the chain's MD substeps in
the frozen fluid with trilinear interpolation and impulse spreading, the
fused collide+stream of every node, the re-collision of the impulse nodes.
Inputs are seeded and synthetic (lbinputs.py) and resident in HBM before the
timed region.  Prints one JSON line.

Default workload: a single 256^3 box (16.8 M nodes, FP32 deviation storage),
chain N = 1024, kT = 1e-4, the box whose step is bound by HBM bandwidth.
Also reported: the 64^3 single box, the 256-box batched sweep against the
same boxes launched box by box, and the dominant kernel against the HBM
roofline.  The oracle is timed on the host cores on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
BYTES_PER_NODE = {0: 304, 1: 152}   # 19 reads + 19 writes of 8 or 4 bytes
KERNEL_SOURCES = ["paper_0903_5067_amd/csrc/lbmd_kernels.hip", "paper_0903_5067_amd/csrc/lbmd_kernels.hpp",
                  "paper_0903_5067_amd/csrc/lbmd_device.hpp"]
PMC_SUMMARY = "profiles/k_collide_prec256_pmc.md"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def make_system(preset, precision=None, n_boxes=None):
    import lbinputs
    import paper_0903_5067_amd as lbm
    P = lbinputs.PRESETS[preset]
    prec = precision if precision is not None else (lbm.FP64 if P["precision"] == "fp64" else lbm.FP32_DEV)
    if preset == "batched256":
        table = lbinputs.batched_table(n_boxes or P["n_boxes"], P["seed"])
        boxes = [lbinputs.box_params(preset, L=L, N=N, box_id=i) for i, (L, N) in enumerate(table)]
    elif preset == "semidilute":
        boxes = [lbinputs.box_params(preset, box_id=i) for i in range(n_boxes or P["n_boxes"])]
    else:
        boxes = [lbinputs.box_params(preset)]
    xs = [lbinputs.initial_chains(b, b["seed"] + 7919 * b["box_id"]) for b in boxes]
    x0 = np.concatenate([x for x in xs if len(x)], axis=0) if any(len(x) for x in xs) else None
    s = lbm.LBSystem(boxes, precision=prec, bead_x0=x0)
    nodes = sum(int(b["L"]) ** 3 for b in boxes)
    return s, boxes, nodes, prec


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(precision_name: str):
    """HBM bytes per collide launch from the committed PMC summary (FETCH_SIZE
    and WRITE_SIZE, each scaled by a plain copy's counter reading), or None
    when there is none for this storage or the kernel sources have changed
    since the counters were taken."""
    path = os.path.join(ROOT, PMC_SUMMARY)
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("traffic:"):
                for kv in line[len("traffic:"):].split():
                    k, _, v = kv.partition("=")
                    vals[k] = v
    if vals.get("source_hash") != kernel_source_hash() or vals.get("precision") != precision_name:
        return None
    try:
        return int(float(vals["bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def copy_calibration():
    """A plain elementwise copy of known size (1 GiB read, 1 GiB written per
    launch, 10 launches) for scaling the HBM byte counters."""
    import torch
    a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.neg(a, out=b)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        torch.neg(a, out=b)
    e1.record()
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / 10
    print(json.dumps({"copy_calibration": {"launches": 11, "read_bytes": a.numel() * 4,
                                           "write_bytes": b.numel() * 4, "kernel": "torch.neg (elementwise)",
                                           "avg_launch_us": round(us, 1),
                                           "gb_per_s": round(2 * a.numel() * 4 / us / 1e3, 1)}}))


def settle(s, seconds):
    """Untimed steps, 20 at a time, until the GPU has been busy `seconds` in
    a row; returns how many ran.  The GPU's clocks drop while it idles (on
    host work, between the autotuner's launches) and take about 0.1 s of load
    to come back, so a short window timed right after an idle spell sees
    them ramping up instead of the sustained rate."""
    n = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        s.step(20)
        s.synchronize()
        n += 20
    return n


def time_steps(s, steps, warmup):
    import torch
    s.step(warmup)
    s.synchronize()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(s.stream)
    s.step(steps)
    e1.record(s.stream)
    s.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / 1e3, wall


def time_collide(s, n):
    """Average duration of the fused collide+stream kernel, HIP events on the
    stream the library launches it on."""
    import torch
    s.collide_only(3)
    s.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s.stream)
    s.collide_only(n)
    e1.record(s.stream)
    s.synchronize()
    return e0.elapsed_time(e1) / 1e3 / n


def thermalization_secondary(L=64, warm=50, samples=300):
    """Node-level mode variances <m_k^2> / (mu rho0 b_k) of a fluid-only 64^3
    box (kT = 1e-2, rates 1.25 / 0.8 / 1.4) with noise on every non-conserved
    mode against noise on the stress modes only (Sec. II.B): group means over
    bulk (k=4), shear (5..9) and ghost (10..18) modes."""
    import lbinputs
    import paper_0903_5067_amd as lbm
    b = np.array([1, 1 / 3, 1 / 3, 1 / 3, 2 / 3, 4 / 3, 4 / 9, 1 / 9, 1 / 9, 1 / 9,
                  2 / 3, 2 / 3, 2 / 3, 2 / 9, 2 / 9, 2 / 9, 2, 4 / 3, 4 / 9])
    out = {}
    for therm, name in ((2, "all_modes"), (1, "stress_only")):
        p = lbinputs.box_params("single64", L=L, N=0, kT=1e-2, therm=therm, omega_s=1.25, omega_b=0.8,
                                omega_g=1.4)
        s = lbm.LBSystem([p], precision=lbm.FP32_DEV)
        s.step(warm)
        acc = np.zeros(19)
        for _ in range(samples):
            s.step(1)
            acc += s.observables()[0]["mode_sq"]
        s.close()
        r = acc / (samples * L ** 3) / (3 * p["kT"] * p["tau_lb"] ** 2 * p["rho0"] * b)
        out[name] = {"bulk": round(float(r[4]), 4), "shear": round(float(np.mean(r[5:10])), 4),
                     "ghost": round(float(np.mean(r[10:])), 4)}
    out["samples"] = samples
    return out


def adjoint_secondary():
    """The 32^3 box with its N=32 chain: a 200-step window with checkpoints
    every 20 steps, forward (recording) and backward (hand-written adjoint)
    timed on the host clock around synchronous library calls, against plain
    steps of the same box."""
    import torch
    import lbinputs
    P = lbinputs.PRESETS["adjoint32"]
    T, k = int(P["steps"]), int(P["checkpoint_every"])
    s, boxes, nodes, prec = make_system("adjoint32")
    tp, _ = time_steps(s, 2000, 50)
    vh = s.window_forward(T, k)          # warm-up, allocates the workspace
    s.window_backward(np.zeros_like(vh))
    s.window_rewind()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    vh = s.window_forward(T, k)
    t1 = time.perf_counter()
    g = s.window_backward(np.cos(np.arange(vh.size)).reshape(vh.shape))
    t2 = time.perf_counter()
    s.close()
    return {"window_steps": T, "checkpoint_every": k, "nodes": nodes, "beads": int(P["N"]),
            "plain_mlups": round(nodes * 2000 / tp / 1e6, 1),
            "forward_ms": round(1e3 * (t1 - t0), 2), "backward_ms": round(1e3 * (t2 - t1), 2),
            "forward_backward_mlups": round(nodes * T / (t2 - t0) / 1e6, 2),
            "grad_finite": bool(np.all(np.isfinite(g)))}


def single64_secondary(graph_steps=20, overlap=True):
    """The 64^3 box with its 64-bead chain: step rate and collide kernel."""
    s64, b64, n64, p64 = make_system("single64")
    s64.set_launch(batched=True, graph_steps=graph_steps, overlap=overlap)
    t64, _ = time_steps(s64, 2000, 50)
    c64 = time_collide(s64, 200)
    o64 = s64.observables()[0]
    s64.close()
    return {"mlups": round(n64 * 2000 / t64 / 1e6, 1), "ms_per_step": round(1e3 * t64 / 2000, 4),
            "collide_us": round(1e6 * c64, 2),
            "collide_gbs": round(BYTES_PER_NODE[p64] * n64 / c64 / 1e9, 1),
            "rg2_after_2050_steps": round(o64["rg2"], 4), "re2_after_2050_steps": round(o64["re2"], 4)}


def batched256_secondary(graph_steps=20, overlap=True):
    """256 boxes of mixed size, one launch per kernel, against the same boxes
    launched box by box."""
    sb, bb, nb, pb = make_system("batched256")
    sb.set_launch(batched=True, graph_steps=graph_steps, overlap=overlap)
    tb, _ = time_steps(sb, 500, 20)
    cb = time_collide(sb, 100)
    sb.set_launch(batched=False)
    tp, _ = time_steps(sb, 100, 5)
    sb.close()
    return {"boxes": len(bb), "nodes": nb, "beads": int(sum(b["N"] for b in bb)),
            "batched_mlups": round(nb * 500 / tb / 1e6, 1),
            "batched_pct_hbm_peak": round(100.0 * BYTES_PER_NODE[pb] * nb * 500 / tb / 1e9 / HBM_PEAK_GBS, 1),
            "plain_per_box_mlups": round(nb * 100 / tp / 1e6, 1),
            "batched_over_plain": round((nb * 500 / tb) / (nb * 100 / tp), 3),
            "collide_us": round(1e6 * cb, 1),
            "collide_gbs": round(BYTES_PER_NODE[pb] * nb / cb / 1e9, 1)}


def semidilute_secondary(steps=300, graph_steps=20):
    """Semidilute solution (Sec. III.C): a batch of 20^3 boxes, each holding 32
    chains of 32 beads (1024 beads, the 1024-thread coupling path), at the
    paper's parameters; against the same boxes holding one 32-bead chain."""
    import lbinputs
    out = {}
    for tag, chains in (("semidilute", None), ("one_chain_per_box", 1)):
        if chains is None:
            s, boxes, nodes, prec = make_system("semidilute")
        else:
            import paper_0903_5067_amd as lbm
            P = lbinputs.PRESETS["semidilute"]
            boxes = [lbinputs.box_params("semidilute", N=32, chain_len=0, box_id=i) for i in range(P["n_boxes"])]
            xs = [lbinputs.initial_chains(b, b["seed"] + 7919 * b["box_id"]) for b in boxes]
            s = lbm.LBSystem(boxes, precision=lbm.FP32_DEV, bead_x0=np.concatenate(xs))
            nodes = sum(int(b["L"]) ** 3 for b in boxes)
        s.set_launch(batched=True, graph_steps=graph_steps)
        t, _ = time_steps(s, steps, 2 * graph_steps)
        obs = s.observables()
        beads = sum(int(b["N"]) for b in boxes)
        sub = int(boxes[0]["md_substeps"])
        out[tag] = {"boxes": len(boxes), "L": int(boxes[0]["L"]),
                    "chains_per_box": int(boxes[0]["N"]) // (int(boxes[0]["chain_len"]) or int(boxes[0]["N"])),
                    "beads_per_box": int(boxes[0]["N"]), "md_substeps": sub,
                    "ms_per_step": round(1e3 * t / steps, 4), "mlups": round(nodes * steps / t / 1e6, 1),
                    "bead_substeps_per_s": round(beads * sub * steps / t, 0),
                    "mean_rg2": round(float(np.mean([o["rg2"] for o in obs])), 3),
                    "health": int(max(o["health"] for o in obs))}
        s.close()
    return out


def cpu_baseline(preset, budget_s=20.0):
    """The oracle (FP64 C, OpenMP) on the host cores: whole LB steps of the
    same box and chain, as many as fit a ~20 s budget (at least one).
    Returns the report and, for the precision study, the oracle's results as
    plain arrays: step count, populations, observables, weights."""
    import tempfile
    import lbinputs
    import oracle
    build_dir = tempfile.mkdtemp(prefix="lbmd_oracle_")
    oracle.use_tuned_build(build_dir)
    p = lbinputs.box_params(preset)
    L = int(p["L"])
    c, w, e, b = oracle.tables()
    n = np.empty((19, L, L, L))
    for i in range(19):
        n[i] = w[i] * p["rho0"]
    x0 = lbinputs.saw_chain(p["N"], L, p["seed"])
    st = oracle.State(oracle.make_box(**p), n, x0)
    del n
    t0 = time.perf_counter()
    st.run(1)
    t1 = time.perf_counter() - t0
    steps = 1
    more = int(max(0, min(50, budget_s / max(t1, 1e-3) - 1)))
    if more:
        t0 = time.perf_counter()
        st.run(more)
        t1 = time.perf_counter() - t0
        steps = more
    mlups = L ** 3 * steps / t1 / 1e6
    cores = oracle.num_threads()
    # one more step on one thread, for the per-core rate
    oracle.set_threads(1)
    t0 = time.perf_counter()
    st.run(1)
    t_one = time.perf_counter() - t0
    oracle.set_threads(cores)
    model = host_cpu()
    rep = {"value": round(mlups, 3), "unit": "MLUPS", "cores": cores, "kind": "oracle",
           "sample": f"{steps} full LB step(s) of the {L}^3 box with its N={p['N']} chain (after 1 untimed), "
                     f"FP64 oracle built g++ {' '.join(oracle.TUNED_FLAGS)} -ffp-contract=off on this host, "
                     f"OpenMP over z-planes, {t1:.1f} s",
           "value_1core": round(L ** 3 / t_one / 1e6, 3), "sample_1core": f"1 further step on 1 thread, {t_one:.1f} s",
           "cpu_model": model}
    oo = st.observables()
    ref = {"t": st.t, "n": st.n, "w": np.array(w),
           "obs": {"mass": oo[0], "p_fluid": oo[4:7], "p_total": oo[10:13], "com": oo[13:16], "rg2": oo[16],
                   "re2": oo[17], "mode_sq": oo[19:38]}}
    return rep, ref


def host_cpu() -> str:
    """The host CPU as lscpu names it (model, family/model/stepping, sockets,
    cores, threads), or /proc/cpuinfo's model name without lscpu."""
    import subprocess
    keep = ("Model name", "Vendor ID", "CPU family", "Model:", "Stepping", "Socket(s)",
            "Core(s) per socket", "Thread(s) per core", "CPU(s):", "CPU max MHz")
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        parts = []
        for line in out.splitlines():
            if line.strip().startswith(keep) and ":" in line:
                k, v = line.split(":", 1)
                parts.append(f"{k.strip()}: {v.strip()}")
        if parts:
            return "; ".join(parts)
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        with open("/proc/cpuinfo") as f:
            return next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        return ""


def _obs_errors(a, b):
    """Per-observable differences of observation dict a from reference b."""
    def rel(x, y):
        return float(abs(x - y) / max(abs(y), 1e-300))
    out = {"mass_rel": rel(a["mass"], b["mass"]),
           "p_total_abs": float(np.max(np.abs(a["p_total"] - b["p_total"]))),
           "p_fluid_abs": float(np.max(np.abs(a["p_fluid"] - b["p_fluid"]))),
           "com_abs": float(np.max(np.abs(a["com"] - b["com"]))),
           "rg2_rel": rel(a["rg2"], b["rg2"]), "re2_rel": rel(a["re2"], b["re2"]),
           "mode_sq_rel_max": float(max(rel(a["mode_sq"][k], b["mode_sq"][k]) for k in range(4, 19)))}
    return {k: float(f"{v:.3e}") for k, v in out.items()}


def precision_study(preset, ref, long_steps):
    """FP32 deviation storage against FP64 storage on the GPU and against the
    oracle's results from the CPU-baseline leg: per-observable differences
    after the oracle's steps (all three from the same initial state and
    noise), and FP32 against FP64 on the GPU after long_steps."""
    import torch
    import paper_0903_5067_amd as lbm
    s_orc, w = ref["t"], ref["w"]
    res = {"short_steps": s_orc, "long_steps": long_steps}
    obs_short = {}
    for prec, name in ((lbm.FP32_DEV, "fp32_dev"), (lbm.FP64, "fp64")):
        s, boxes, nodes, _ = make_system(preset, precision=prec)
        s.set_launch(batched=True, graph_steps=20)
        s.step(s_orc)
        ob = s.observables()[0]
        obs_short[name] = ob
        n = s.export_state()["boxes"][0]["n"]
        err = 0.0
        for i in range(19):
            err = max(err, float(np.max(np.abs(n[i] - ref["n"][i]))) / (w[i] * boxes[0]["rho0"]))
        del n
        e_o = _obs_errors(ob, ref["obs"])
        e_o["pop_rel_max"] = float(f"{err:.3e}")
        res[f"{name}_vs_oracle"] = e_o
        t_long, _ = time_steps(s, long_steps - s_orc, 0)
        obs_short[name + "_long"] = s.observables()[0]
        t_k = time_collide(s, 100)
        res[f"{name}_step_mlups"] = round(nodes * (long_steps - s_orc) / t_long / 1e6, 1)
        res[f"{name}_collide_us"] = round(t_k * 1e6, 1)
        res[f"{name}_collide_gbs"] = round(BYTES_PER_NODE[prec] * nodes / t_k / 1e9, 1)
        s.close()
        del s
        torch.cuda.empty_cache()
    res["fp32_dev_vs_fp64_gpu_short"] = _obs_errors(obs_short["fp32_dev"], obs_short["fp64"])
    res["fp32_dev_vs_fp64_gpu_long"] = _obs_errors(obs_short["fp32_dev_long"], obs_short["fp64_long"])
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="prec256", choices=["prec256", "single64", "plain16"])
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--graph-steps", type=int, default=20)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--settle", type=float, default=0.25,
                    help="seconds of untimed steps before the warm-up steps, so that the timed steps "
                         "run at sustained clocks (0: --warmup steps only)")
    ap.add_argument("--variant", type=int, default=-1,
                    help="force this collide launch shape instead of autotuning")
    ap.add_argument("--collide-launches", type=int, default=0,
                    help="launches of the collide kernel timed for the roofline (0: ~0.5 s worth)")
    ap.add_argument("--fixup-after-collide", action="store_true",
                    help="re-collide the chain's nodes after the collide instead of colliding their tiles "
                         "beside it (same results; for comparison)")
    ap.add_argument("--no-resident-wait", action="store_true",
                    help="no chain kernel waits for a later collide (needed under hardware counter "
                         "collection, which runs one kernel at a time)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run the plain copy used to scale the HBM byte counters")
    ap.add_argument("--only-semidilute", action="store_true",
                    help="only run the semidilute secondary and print it")
    ap.add_argument("--only-single64", action="store_true",
                    help="only run the 64^3 secondary and print it")
    ap.add_argument("--only-batched256", action="store_true",
                    help="only run the 256-box secondary and print it")
    ap.add_argument("--only-adjoint", action="store_true",
                    help="only run the adjoint-window secondary and print it")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the path is built and measured for a single MI355X; "
              "multi-GPU sharding is a design note, not part of this build", file=sys.stderr)
        sys.exit(2)

    import torch
    import lbinputs
    torch.cuda.init()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.only_semidilute:
        print(json.dumps(semidilute_secondary()), flush=True)
        return
    if args.only_single64:
        print(json.dumps(single64_secondary(args.graph_steps, not args.fixup_after_collide)), flush=True)
        return
    if args.only_batched256:
        print(json.dumps(batched256_secondary(args.graph_steps, not args.fixup_after_collide)), flush=True)
        return
    if args.only_adjoint:
        print(json.dumps(adjoint_secondary()), flush=True)
        return
    log("workload", args.workload)
    s, boxes, nodes, prec = make_system(args.workload)
    if args.graph_steps or args.fixup_after_collide or args.no_resident_wait:
        s.set_launch(batched=True, graph_steps=args.graph_steps, overlap=not args.fixup_after_collide,
                     resident=not args.no_resident_wait)
    tune = None
    import paper_0903_5067_amd as lbm
    if args.variant >= 0:
        s.set_collide_variant(args.variant)
        tune = {"chosen": args.variant, "shape": lbm.COLLIDE_VARIANT_SHAPES[args.variant], "forced": True}
    elif not args.no_autotune:
        chosen, times = s.autotune(reps=20)
        tune = {"chosen": chosen, "shape": lbm.COLLIDE_VARIANT_SHAPES[chosen],
                "us_per_variant": [round(t, 2) for t in times]}
        log("autotune", json.dumps(tune))
    obs0 = s.observables()[0]
    n_settle = settle(s, args.settle)
    t_ev, t_wall = time_steps(s, args.steps, args.warmup)
    obs1 = s.observables()[0]
    ms = 1e3 * t_ev / args.steps
    mlups = nodes * args.steps / t_ev / 1e6
    log(f"{args.steps} steps: {t_ev:.4f} s (events), {t_wall:.4f} s (wall), {mlups:.1f} MLUPS")
    n_coll = args.collide_launches or max(20, min(500, int(2.0 / max(ms / 1e3, 1e-6) / 4)))
    t_k = time_collide(s, n_coll)
    achieved = BYTES_PER_NODE[prec] * nodes / t_k / 1e9
    log(f"collide kernel: {t_k * 1e6:.1f} us avg over {n_coll} launches, {achieved:.0f} GB/s")
    P = lbinputs.PRESETS[args.workload]
    result = {
        "metric": "LB node updates/s (MLUPS) + % HBM peak",
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "settle_steps": n_settle,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == 1 else "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: single {P['L']}^3 periodic box, chain N={P['N']}, "
                               f"kT={P['kT']}, {'FP32 deviation' if prec == 1 else 'FP64'} populations, "
                               f"{P['md_substeps']} MD substeps per LB step",
                   "nodes": nodes, "beads": int(P["N"]), "precision": "fp32_dev" if prec == 1 else "fp64"},
        "pct_hbm_peak_step": round(100.0 * BYTES_PER_NODE[prec] * nodes * args.steps / t_ev / 1e9 / HBM_PEAK_GBS, 2),
        "roofline": {"bound": "hbm", "kernel": "k_collide (fused collide+stream)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": (measured_traffic("fp32_dev" if prec == 1 else "fp64")
                                 if args.workload == "prec256" else None),
                     "bytes_per_launch": BYTES_PER_NODE[prec] * nodes,
                     "avg_launch_us": round(t_k * 1e6, 2)},
        "autotune": tune,
        "invariants": {"mass_rel_drift": abs(obs1["mass"] - obs0["mass"]) / obs0["mass"],
                       "p_total_drift": float(np.max(np.abs(obs1["p_total"] - obs0["p_total"]))),
                       "health": obs1["health"]},
    }
    s.close()
    del s
    torch.cuda.empty_cache()

    if not args.no_secondary:
        sec = {}
        sec["single64"] = single64_secondary(args.graph_steps, not args.fixup_after_collide)
        sec["batched256"] = batched256_secondary(args.graph_steps, not args.fixup_after_collide)
        sec["adjoint32"] = adjoint_secondary()
        sec["thermalization"] = thermalization_secondary()
        sec["semidilute"] = semidilute_secondary()
        result["secondary"] = sec
        log("secondary", json.dumps(sec))
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        rep, ref = cpu_baseline(args.workload)
        result["cpu_baseline"] = rep
        if args.workload == "prec256" and not args.no_secondary:
            log("precision study ...")
            result["precision"] = precision_study(args.workload, ref, 2000)
            log("precision", json.dumps(result["precision"]))
        del ref
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
