#!/usr/bin/env python3
"""Throughput of the per-particle Lagrangian step on one MI355X.

Workload: curved sine-mapped periodic box with curved reflective walls,
32^3 hexahedra of geometry degree 4, DG degree 5 random-Fourier fluid state,
1e6 particles, Schiller-Naumann drag, 3-stage low-storage RK, dt = 1e-3, FP64.
One timed step = one fp_step(dt, 1): counting sort by element, then three fused
RK-stage launches (guess, Newton, interpolation, drag, update, tracking with
face intersection, hand-off and wall reflection, inside verification).

Prints one JSON line.  Also measured: the mixed-precision form (FP32 fluid
state, FP32 interpolation/drag/RK) with its position error against the FP64
form, the dominant kernel against its roofline, and the FP64 CPU oracle on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6      # MI355X vector FP64
PEAK_HBM_GBS = 8000.0        # MI355X HBM3E
# the stage kernel's sources and its compile flags
KERNEL_SOURCES = ["paper_2211_05458_amd/csrc/fp_device.h", "paper_2211_05458_amd/csrc/stage.hip",
                  "paper_2211_05458_amd/csrc/fp_internal.h", "paper_2211_05458_amd/build.py"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_stage_elem_fp64_curved32_traffic.md")


def stage_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic():
    """Per-launch HBM bytes of the stage kernel from the committed counter summary,
    only if it was taken on the current kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    for line in open(TRAFFIC_FILE):
        if line.startswith("source_hash:"):
            vals["hash"] = line.split(":", 1)[1].strip()
        if line.startswith("hbm_bytes_per_launch:"):
            vals["bytes"] = float(line.split(":", 1)[1].strip())
    if vals.get("hash") != stage_source_hash() or "bytes" not in vals:
        return None
    return vals["bytes"]


# variables the drag law reads (density, momentum); the energy is not needed
INTERP_VARS = 4


def flops_per_particle_stage(n, ng, newton_it):
    """Algorithmic flops of one particle-stage: Newton iterations on the
    geometry map and Jacobian (sum factorisation), interpolation of the drag
    law's variables, the nearest-node guess, and the drag, update and box
    tests."""
    f_newton = 6 * (2 * ng ** 3 + 3 * ng ** 2 + 4 * ng) + 160
    f_interp = 2 * INTERP_VARS * (n ** 3 + n ** 2 + n) + 9 * n ** 2
    f_guess = 8 * ng ** 3
    f_rest = 300
    return newton_it * f_newton + f_interp + f_guess + f_rest


def bytes_per_particle_stage(n, ng, ppe):
    """Algorithmic HBM bytes of one particle-stage, FP64 state: particle SoA read
    (x, v, kx, kv, d, elem, status) and write (x, v, kx, kv, elem), plus the
    element's fluid state (the variables read), geometry and face records amortised
    over its particles."""
    soa = (12 * 8 + 8 + 4 + 1) + (12 * 8 + 4)
    elem = INTERP_VARS * n ** 3 * 8 + 3 * ng ** 3 * 8 + 336
    return soa + elem / ppe


def run_gpu(w, U, precision, steps, warmup, guess=0, weights=None, deposit=None, keep=False, tracking=0, forces=0,
            gravity=(0.0, 0.0, 0.0), sort_every=1):
    """Push w's particles, run `warmup` untimed then `steps` timed fp_step(dt, 1)
    calls (each followed by deposit(g) if given); returns timings and the state."""
    import numpy as np
    import torch
    from paper_2211_05458_amd.lib import FlexiPart
    g = FlexiPart(w.mesh, w.N, w.n_particles)
    g.set_fluid_state(U)
    st, nrej = g.push(w.x, w.v, w.d, w.elem_hint)
    n_active = int((st == 0).sum())
    n_flagged = g.mlp_set_weights(weights) if weights is not None else 0
    opts = dict(rk=w.rk, drag=w.drag, precision=precision, sort_every=sort_every, guess=guess, tracking=tracking,
                forces=forces, gravity=gravity)
    for _ in range(warmup):
        g.step(w.dt, 1, **opts)
        if deposit:
            deposit(g)
    torch.cuda.synchronize()
    g.reset_stats()
    g.timing()
    g.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(steps):
        g.step(w.dt, 1, **opts)
        if deposit:
            deposit(g)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1)
    timing = g.timing()
    g.set_timing(False)
    stats = g.stats()
    r = g.read()
    out = dict(ms=ms, wall=wall, timing=timing, stats=stats, read=r, n_active=n_active, n_flagged=n_flagged,
               active_end=int((r["status"] == 0).sum()),
               kernel_ms={k: (v[1] / v[0] if v[0] else 0.0) for k, v in timing.items()})
    if keep:
        out["ctx"] = g
    else:
        g.close()
    return out


def pos_error(ref, other, h):
    """Position difference of two runs from the same initial state."""
    import numpy as np
    both = (ref["read"]["status"] == 0) & (other["read"]["status"] == 0)
    dx = np.linalg.norm(other["read"]["x"][both] - ref["read"]["x"][both], axis=1)
    return {"pos_err_max_m": float(dx.max()), "pos_err_rms_m": float(np.sqrt((dx ** 2).mean())),
            "pos_err_max_h": float(dx.max() / h),
            "elem_mismatch_frac": float((other["read"]["elem"] != ref["read"]["elem"]).mean()),
            "hits_mismatch_frac": float((other["read"]["hits"] != ref["read"]["hits"]).mean())}


def summary(r, K):
    return {"value": r["n_active"] * K / (r["ms"] * 1e-3), "ms_per_step": r["ms"] / K,
            "kernel_ms": r["kernel_ms"],
            "newton_it_per_solve": r["stats"]["newton_iters"] / max(r["stats"]["newton_calls"], 1),
            "fallbacks": r["stats"]["fallbacks"], "lost": r["stats"]["lost"]}


def bench_annulus(args):
    """Annular-sector passage 48x24x48, Ngeo=6, N=5: plain FP64 against the
    mixed form with the learned Newton guess trained on the GPU."""
    import numpy as np
    import torch
    from paper_2211_05458_amd import workloads as W
    from paper_2211_05458_amd.lib import FlexiPart
    n = args.particles or 10_000_000
    K, Wm = args.steps or 10, args.warmup
    print("[bench] generating annulus workload", file=sys.stderr, flush=True)
    w = W.config4(n_particles=n)
    U64 = torch.from_numpy(w.U).cuda()
    U32 = torch.from_numpy(w.U.astype(np.float32)).cuda()
    print("[bench] training pairs and training", file=sys.stderr, flush=True)
    n_train = min(n, 1_000_000)
    t0 = time.perf_counter()
    g = FlexiPart(w.mesh, w.N, n_train)
    g.set_fluid_state(U64)
    g.push(w.x[:n_train], w.v[:n_train], w.d[:n_train], w.elem_hint[:n_train])
    feat, xi = g.newton_pairs()
    wts, hist = g.mlp_train(feat, xi, epochs=args.epochs, batch=1024, lr=2e-3, seed=4)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    pred = g.mlp_forward(wts, feat)
    guess_err = float((pred - xi).abs().max(dim=1).values.median().item())
    g.close()
    runs = {}
    for name, U, prec, guess, tr in [("fp64", U64, 0, 0, 0), ("fp64_learned", U64, 0, 1, 0), ("mixed", U32, 1, 0, 0),
                                     ("mixed_learned", U32, 1, 1, 0), ("mixed_learned_refspace", U32, 1, 1, 1)]:
        print("[bench] run", name, file=sys.stderr, flush=True)
        runs[name] = run_gpu(w, U, prec, K, Wm, guess=guess, weights=wts if guess else None, tracking=tr)
    out = {"metric": "particle-steps/sec/GPU (plain FP64 vs FP32+MLP-guess) at stated position error",
           "value": summary(runs["mixed_learned"], K)["value"], "unit": "particle-steps/s", "n_gpus": 1,
           "steps": K, "warmup": Wm, "higher_is_better": True, "dtype": "f32+f64", "data": "synthetic",
           "config": {"workload": "annular passage 48x24x48 Ngeo=6, DG N=5, %d particles, Schiller-Naumann, "
                                  "3-stage LSERK, dt=1e-3" % n, "elements": w.mesh.n_elem},
           "training": {"pairs": int(feat.shape[0]), "epochs": args.epochs, "batch": 1024, "seconds": train_s,
                        "loss_first_epoch": hist[0], "loss_last_epoch": hist[-1],
                        "median_guess_error": guess_err, "flagged_elements": runs["fp64_learned"]["n_flagged"]}}
    for k, r in runs.items():
        out[k] = summary(r, K)
        if k != "fp64":
            out[k].update(pos_error(runs["fp64"], r, w.mesh.h))
    out["speedup_mixed_learned_vs_fp64"] = out["mixed_learned"]["value"] / out["fp64"]["value"]
    out["speedup_mixed_learned_refspace_vs_fp64"] = out["mixed_learned_refspace"]["value"] / out["fp64"]["value"]
    print(json.dumps(out))


def bench_precision(args):
    """64^3 curved box, Ngeo=4, N=7, FP32 fluid state: FP64 against mixed."""
    import numpy as np
    import torch
    from paper_2211_05458_amd import workloads as W
    n = args.particles or 10_000_000
    K, Wm = args.steps or 10, args.warmup
    print("[bench] generating 64^3 N=7 workload", file=sys.stderr, flush=True)
    w = W.config3(n_particles=n)
    U64 = torch.from_numpy(w.U).cuda()
    U32 = torch.from_numpy(w.U.astype(np.float32)).cuda()
    del w.U
    r64 = run_gpu(w, U64, 0, K, Wm)
    del U64
    r32 = run_gpu(w, U32, 1, K, Wm)
    out = {"metric": "particle-steps/sec/GPU (plain FP64 vs FP32+MLP-guess) at stated position error",
           "value": summary(r32, K)["value"], "unit": "particle-steps/s", "n_gpus": 1, "steps": K, "warmup": Wm,
           "higher_is_better": True, "dtype": "f32+f64", "data": "synthetic",
           "config": {"workload": "curved sine box 64^3 Ngeo=4, DG N=7 (fluid state FP32), %d particles, "
                                  "Schiller-Naumann, 3-stage LSERK, dt=1e-3" % n, "elements": w.mesh.n_elem},
           "fp64": summary(r64, K), "mixed": summary(r32, K)}
    out["mixed"].update(pos_error(r64, r32, w.mesh.h))
    out["mixed"]["after_steps"] = K + Wm
    out["speedup_mixed_vs_fp64"] = out["mixed"]["value"] / out["fp64"]["value"]
    print(json.dumps(out))


def bench_twoway(args):
    """96^3 curved box, Ngeo=4, N=5, 2e7 particles, mixed form, shape-kernel
    source (R = 1.5 h) deposited after every step."""
    import numpy as np
    import torch
    from paper_2211_05458_amd import workloads as W
    n = args.particles or 20_000_000
    K, Wm = args.steps or 5, min(args.warmup, 2)
    print("[bench] generating 96^3 workload", file=sys.stderr, flush=True)
    w = W.config5(n_particles=n)
    U32 = torch.from_numpy(w.U.astype(np.float32)).cuda()
    del w.U
    R = 1.5 * w.mesh.h
    per = np.array([1.0, 0.0, 1.0])
    S = {}

    def dep(g):
        if "S" not in S:
            S["S"] = torch.zeros((g.E, 4, g.n3), dtype=torch.float32, device="cuda")
        S["S"].zero_()
        g.deposit(S["S"], kind=1, radius=R, period=per)

    r = run_gpu(w, U32, 1, K, Wm, deposit=dep, keep=True)
    g = r["ctx"]
    V = g.node_volumes()
    tot_shape = (S["S"].double() * V[:, None, :]).sum(dim=(0, 2))
    Sn = g.deposit(None, kind=0, dtype=torch.float64)
    tot_near = (Sn * V[:, None, :]).sum(dim=(0, 2))
    cons = float(((tot_shape - tot_near).abs().max() / tot_near.abs().max()).item())
    out = {"metric": "particle-steps/sec/GPU (plain FP64 vs FP32+MLP-guess) at stated position error",
           "value": summary(r, K)["value"], "unit": "particle-steps/s", "n_gpus": 1, "steps": K, "warmup": Wm,
           "higher_is_better": True, "dtype": "f32+f64", "data": "synthetic",
           "config": {"workload": "curved sine box 96^3 Ngeo=4, DG N=5, %d particles, mixed form, shape-kernel "
                                  "two-way source R=1.5h every step" % n, "elements": w.mesh.n_elem},
           "run": summary(r, K),
           "conservation_rel_err_fp32": cons,
           "deposited_momentum": [float(v) for v in tot_near[:3].tolist()]}
    print(json.dumps(out))


def bench_mortar(args):
    """Non-conforming mesh: a coarse block of 16^3 curved elements (Ngeo=4)
    against a fine block refined 4:1 across the interface (16x32x32), DG N=5,
    walls all round, 1e6 particles, FP64.  Every coarse face on the interface
    is a big mortar face."""
    import numpy as np
    import torch
    from paper_2211_05458_amd import workloads as W
    n = args.particles or 1_000_000
    K, Wm = args.steps or 100, args.warmup
    print("[bench] generating mortar workload", file=sys.stderr, flush=True)
    w = W.mortar_box(n_geo=4, N=5, refine=(2, 2), n_particles=n, cells=(16, 16, 16), seed=1006)
    U64 = torch.from_numpy(w.U).cuda()
    runs = {}
    for name, tr in (("fp64", 0), ("fp64_refspace", 1)):
        print("[bench] run", name, file=sys.stderr, flush=True)
        runs[name] = run_gpu(w, U64, 0, K, Wm, tracking=tr)
    out = {"metric": "particle-steps/sec/GPU (plain FP64 vs FP32+MLP-guess) at stated position error",
           "value": summary(runs["fp64"], K)["value"], "unit": "particle-steps/s", "n_gpus": 1, "steps": K,
           "warmup": Wm, "higher_is_better": True, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "non-conforming box: 16^3 coarse + 16x32x32 fine curved elements (4:1 mortar "
                                  "interface, %d big faces), Ngeo=4, DG N=5, %d particles, Schiller-Naumann, "
                                  "3-stage LSERK, dt=1e-3, FP64" % (len(w.mesh.mortar), n),
                      "elements": w.mesh.n_elem}}
    for k, r in runs.items():
        out[k] = summary(r, K)
        out[k].update({"crossings": r["stats"]["crossings"], "wall_hits": r["stats"]["wall_hits"],
                       "recovered": r["stats"]["recovered"], "active_end": r["active_end"]})
    out["fp64_refspace"].update(pos_error(runs["fp64"], runs["fp64_refspace"], w.mesh.h))
    print(json.dumps(out))


def copy_calibration(gib=2, reps=5):
    """Device-to-device copy of a known byte count (counter calibration)."""
    import torch
    n = gib * (1 << 30) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "reps": reps}))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--particles", type=int, default=None)
    ap.add_argument("--workload", choices=["curved32", "annulus", "precision", "twoway", "mortar"], default="curved32",
                    help="curved32: the benchmark line; the others measure the remaining workloads")
    ap.add_argument("--epochs", type=int, default=20, help="learned-guess training epochs (annulus)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-refspace", action="store_true", help="skip the reference-space localisation run")
    ap.add_argument("--no-forces", action="store_true", help="skip the extra-forces run")
    ap.add_argument("--sort-every", type=int, default=1, help="counting sort by element every k steps")
    ap.add_argument("--cpu-every", type=int, default=2, help="oracle sample: every k-th particle")
    ap.add_argument("--cpu-steps", type=int, default=30)
    ap.add_argument("--mode", choices=["bench", "copy"], default="bench",
                    help="copy: a plain device copy of known size, the calibration for HBM counters")
    args = ap.parse_args()
    if args.mode == "copy":
        copy_calibration()
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    from paper_2211_05458_amd import workloads as W
    W.VERBOSE = True
    if args.workload != "curved32":
        {"annulus": bench_annulus, "precision": bench_precision, "twoway": bench_twoway,
         "mortar": bench_mortar}[args.workload](args)
        return
    args.steps = args.steps or 100
    args.particles = args.particles or 1_000_000

    import numpy as np
    import torch
    from paper_2211_05458_amd import workloads as W

    print("[bench] generating workload", file=sys.stderr, flush=True)
    w = W.config2(n_particles=args.particles)
    n, ng = w.N + 1, w.mesh.n_geo + 1
    U64 = torch.from_numpy(w.U).cuda()
    print("[bench] FP64 run", file=sys.stderr, flush=True)
    r64 = run_gpu(w, U64, 0, args.steps, args.warmup, sort_every=args.sort_every)
    K = args.steps
    value = r64["n_active"] * K / (r64["ms"] * 1e-3)
    stages = 3
    n_launch, stage_ms = r64["timing"]["stage_elem"]
    sort_launch, sort_ms = r64["timing"]["sort"]
    avg_stage_ms = stage_ms / max(n_launch, 1)
    ps = r64["n_active"] * stages * K                       # particle-stages timed
    it_per_ps = r64["stats"]["newton_iters"] / ps
    fl_ps = flops_per_particle_stage(n, ng, it_per_ps)
    ppe = r64["n_active"] / w.mesh.n_elem
    by_ps = bytes_per_particle_stage(n, ng, ppe)
    # particles handled by the element-wise kernel per launch (the rest left
    # their sorted element and go through the per-lane kernel)
    per_launch_particles = (ps - r64["stats"]["stragglers"]) / max(n_launch, 1)
    per_launch_flops = fl_ps * per_launch_particles
    per_launch_bytes = by_ps * per_launch_particles
    kern_ms = r64["kernel_ms"]
    achieved_tf = per_launch_flops / (avg_stage_ms * 1e-3) / 1e12
    achieved_gbs = per_launch_bytes / (avg_stage_ms * 1e-3) / 1e9
    traffic = read_traffic()

    extras = {}
    if not args.no_mixed:
        print("[bench] mixed-precision run", file=sys.stderr, flush=True)
        U32 = torch.from_numpy(w.U.astype(np.float32)).cuda()
        r32 = run_gpu(w, U32, 1, args.steps, args.warmup)
        extras["mixed_fp32"] = summary(r32, K)
        extras["mixed_fp32"].update(pos_error(r64, r32, w.mesh.h))
        extras["mixed_fp32"].update({
            "after_steps": args.warmup + K,
            "learned_guess": "no element of this mesh deviates from its trilinear corner map by "
                             "more than 0.05 h, so the learned guess is never used here",
        })

    if not args.no_refspace:
        # the paper's reference-space localisation: segments that cannot reach a
        # wall or periodic face are localised by Newton instead of traced
        print("[bench] reference-space localisation run", file=sys.stderr, flush=True)
        rr = run_gpu(w, U64, 0, args.steps, args.warmup, tracking=1)
        extras["fp64_refspace"] = summary(rr, K)
        extras["fp64_refspace"].update(pos_error(r64, rr, w.mesh.h))
        extras["fp64_refspace"].update({"crossings_traced": rr["stats"]["crossings"],
                                        "localised": rr["stats"]["recovered"],
                                        "track_queue": rr["stats"]["track_queue"]})

    if not args.no_forces:
        # the extra terms of the equation of motion (buoyancy, undisturbed-flow
        # stress, added mass, Saffman lift) with gravity; they run through the
        # per-lane stage kernel
        print("[bench] extra-forces run", file=sys.stderr, flush=True)
        rf = run_gpu(w, U64, 0, args.steps, args.warmup, forces=15, gravity=(0.0, -9.81, 0.0))
        extras["fp64_forces"] = summary(rf, K)
        extras["fp64_forces"].update({"forces": "buoyancy+stress+added_mass+saffman", "gravity": [0.0, -9.81, 0.0]})

    cpu = None
    if not args.no_cpu_baseline:
        import oracle as O
        print("[bench] CPU oracle sample", file=sys.stderr, flush=True)
        idx = np.arange(0, w.n_particles, args.cpu_every)
        o = O.Oracle(w.mesh, w.N, w.U)
        o.push(w.x[idx], w.v[idx], w.d[idx], w.elem_hint[idx])
        t0 = time.perf_counter()
        o.step(w.dt, args.cpu_steps, rk=w.rk, drag=w.drag)
        el = time.perf_counter() - t0
        cpu = {"value": len(idx) * args.cpu_steps / el, "unit": "particle-steps/s", "cores": O.num_threads(),
               "kind": "oracle",
               "sample": "one particle in %d (%d of %d) for %d steps of the same workload, FP64, "
                         "%.1f s wall" % (args.cpu_every, len(idx), w.n_particles, args.cpu_steps, el)}
        # the same oracle on one core, over a sixteenth of that sample
        n_all = O.num_threads()
        idx1 = idx[::16]
        o1 = O.Oracle(w.mesh, w.N, w.U)
        o1.push(w.x[idx1], w.v[idx1], w.d[idx1], w.elem_hint[idx1])
        O.set_num_threads(1)
        t0 = time.perf_counter()
        o1.step(w.dt, args.cpu_steps, rk=w.rk, drag=w.drag)
        el1 = time.perf_counter() - t0
        O.set_num_threads(n_all)
        cpu.update({"value_1core": len(idx1) * args.cpu_steps / el1,
                    "sample_1core": "%d particles for %d steps on one thread, %.1f s wall" % (len(idx1), args.cpu_steps,
                                                                                         el1)})

    out = {
        "metric": "particle-steps/sec/GPU (plain FP64 vs FP32+MLP-guess) at stated position error",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": r64["ms"] / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "curved sine box 32^3 Ngeo=4, DG N=5 random-Fourier state, %d particles, "
                               "Schiller-Naumann, 3-stage LSERK, dt=1e-3, FP64, one-way" % w.n_particles,
                   "elements": w.mesh.n_elem, "particles": w.n_particles, "N": w.N, "n_geo": w.mesh.n_geo},
        "roofline": {"bound": "alu", "achieved": achieved_tf, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved_tf / PEAK_FP64_TFLOPS, "traffic": traffic,
                     "kernel": "k_stage_elem<6,5,double,false,false,false>", "avg_launch_ms": avg_stage_ms,
                     "particles_per_launch": per_launch_particles,
                     "flops_per_particle_stage": fl_ps, "newton_it_per_particle_stage": it_per_ps,
                     "algorithmic_bytes_per_launch": per_launch_bytes,
                     "algorithmic_GBs": achieved_gbs, "hbm_frac": achieved_gbs / PEAK_HBM_GBS},
        "kernel_ms": kern_ms,
        "stats": r64["stats"],
        "cpu_baseline": cpu,
    }
    out.update(extras)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
