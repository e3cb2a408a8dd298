#!/usr/bin/env python3
"""Throughput of the per-particle Lagrangian step on one MI355X.

Default line (the largest single-GPU workload): two-way coupling at scale, a
96^3 curved sine box of geometry degree 4, DG degree 5 random-Fourier state,
2e7 particles, Schiller-Naumann drag, 3-stage low-storage RK, dt = 1e-3, and
the polynomial shape-kernel source (R = 1.5 h) deposited after every step.
One timed step = one fp_step(dt, 1) (counting sort, three stage launches:
guess, Newton, interpolation, drag, update, tracking) plus the zeroed source
and one fp_deposit_source.  `value` is the FP32 + learned-guess form (FP32
interpolation, drag and update, FP64 Newton tail and tracking, the learned
Newton guess on strongly curved elements, FP32 source on the matrix cores);
the plain FP64 form (FP64 throughout, FP64 source) runs beside it.  A second
leg compares the same forms on the annular passage (geometry degree 6, 1e7
particles), where the learned guess acts.  Every leg states its position
error against the FP64 oracle after the workload's full step count on a
fixed subset of its particles, and carries the roofline of its dominant
kernel; cpu_baseline times the oracle on a bounded sample.

Other workloads for manual runs: --workload curved32 | annulus | precision |
twoway | mortar; --mode copy is the calibration of the HBM counters.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6      # MI355X vector FP64 (and unpacked FP32 vector)
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
METRIC = "particle-steps/sec/GPU (plain FP64 vs FP32+MLP-guess) at stated position error"
INTERP_VARS = 4              # variables the drag law reads (density, momentum)
# algorithmic flops per (particle, node) pair within R of the shape-kernel
# source: |x_n - x_p|^2 (8), 1 - r^2/R^2 (2), K = q^2 (1), then K V summed
# (2, normalisation pass) or K G for four components (8, node-sum pass)
DEP_FLOPS_NORM = 13
DEP_FLOPS_GATHER = 19
TRAFFIC = {   # committed counter summaries: kernel -> (file, sources its hash covers)
    "k_dep_norm_mfma": ("profiles/k_dep_norm_mfma_twoway96_traffic.md",
                        ["paper_2211_05458_amd/csrc/deposit.hip", "paper_2211_05458_amd/build.py"]),
    "k_dep_gather_mfma": ("profiles/k_dep_gather_mfma_twoway96_traffic.md",
                          ["paper_2211_05458_amd/csrc/deposit.hip", "paper_2211_05458_amd/build.py"]),
}


# the annular passage's small, strongly curved elements: about a tenth of the
# particles cross a face in each stage, so every form there sorts before every
# stage and runs those particles in their new element's task (bitwise the same
# results as the per-lane kernel)
ANNULUS_SORT = -1

# guess bit 1 in every form: each particle is located from its reference
# coordinates of the previous stage continued along its displacement first
# (the paper's guess after a crossing or reflection); --no-warm turns it off
WARM = 2


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def source_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(kernel):
    """HBM bytes per launch of `kernel` from its committed counter summary, only
    if the summary was taken on the current kernel sources (else None)."""
    if kernel not in TRAFFIC:
        return None
    path, files = TRAFFIC[kernel]
    path = os.path.join(ROOT, path)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if line.startswith("source_hash:"):
            vals["hash"] = line.split(":", 1)[1].strip()
        if line.startswith("hbm_bytes_per_launch:"):
            vals["bytes"] = float(line.split(":", 1)[1].strip())
    if vals.get("hash") != source_hash(files) or "bytes" not in vals:
        return None
    return vals["bytes"]


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


# ---------------------------------------------------------------------------
# algorithmic work per unit
# ---------------------------------------------------------------------------
def flops_per_particle_stage(n, ng, newton_it):
    """Newton iterations on the geometry map and Jacobian (sum factorisation),
    interpolation of the drag law's variables, the nearest-node guess, and the
    drag, update and box tests."""
    f_newton = 6 * (2 * ng ** 3 + 3 * ng ** 2 + 4 * ng) + 160
    f_interp = 2 * INTERP_VARS * (n ** 3 + n ** 2 + n) + 9 * n ** 2
    f_guess = 8 * ng ** 3
    return newton_it * f_newton + f_interp + f_guess + 300


def bytes_per_particle_stage(n, ng, ppe, ubytes=8):
    """Particle SoA read (x, v, kx, kv, d, elem, status) and write (x, v, kx, kv,
    elem), plus the element's fluid state (the variables read), geometry and
    face records amortised over its particles."""
    soa = (12 * 8 + 8 + 4 + 1) + (12 * 8 + 4)
    return soa + (INTERP_VARS * n ** 3 * ubytes + 3 * ng ** 3 * 8 + 336) / ppe


# ---------------------------------------------------------------------------
# GPU runs
# ---------------------------------------------------------------------------
def run_gpu(w, U, precision, steps, warmup, guess=0, weights=None, deposit=None, keep=False, tracking=0, forces=0,
            gravity=(0.0, 0.0, 0.0), sort_every=1, idx=None):
    """Push w's particles (or the subset idx), run `warmup` untimed then `steps`
    timed fp_step(dt, 1) calls, each followed by deposit(g) if given."""
    import numpy as np
    import torch
    from paper_2211_05458_amd.lib import FlexiPart
    x, v, d, h = (w.x, w.v, w.d, w.elem_hint) if idx is None else (w.x[idx], w.v[idx], w.d[idx], w.elem_hint[idx])
    g = FlexiPart(w.mesh, w.N, len(x))
    g.set_fluid_state(U)
    st, nrej = g.push(x, v, d, h)
    n_active = int((st == 0).sum())
    n_flagged = g.mlp_set_weights(weights) if weights is not None else 0
    opts = dict(rk=w.rk, drag=w.drag, precision=precision, sort_every=sort_every, guess=guess | WARM,
                tracking=tracking, forces=forces, gravity=gravity)
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


def summary(r, K):
    return {"value": r["n_active"] * K / (r["ms"] * 1e-3), "ms_per_step": r["ms"] / K,
            "kernel_ms": {k: round(v, 4) for k, v in r["kernel_ms"].items() if v > 0},
            "newton_it_per_solve": r["stats"]["newton_iters"] / max(r["stats"]["newton_calls"], 1),
            "fallbacks": r["stats"]["fallbacks"], "lost": r["stats"]["lost"]}


def stage_roofline(r, w, K, stages, ubytes=8):
    """k_stage_elem: algorithmic flops (and bytes) of the particle-stages it
    processed per launch, over its live HIP-event average."""
    n, ng = w.N + 1, w.mesh.n_geo + 1
    n_launch, tot_ms = r["timing"]["stage_elem"]
    if not n_launch:
        return None
    avg = tot_ms / n_launch
    ps = r["n_active"] * stages * K
    it = r["stats"]["newton_iters"] / max(ps, 1)
    per_launch = (ps - r["stats"]["stragglers"]) / n_launch
    fl = flops_per_particle_stage(n, ng, it) * per_launch
    by = bytes_per_particle_stage(n, ng, r["n_active"] / w.mesh.n_elem, ubytes) * per_launch
    ach = fl / (avg * 1e-3) / 1e12
    return {"bound": "alu", "achieved": ach, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
            "frac": ach / PEAK_FP64_TFLOPS, "traffic": None, "kernel": "k_stage_elem", "avg_launch_ms": avg,
            "particles_per_launch": per_launch, "newton_it_per_particle_stage": it,
            "algorithmic_bytes_per_launch": by, "hbm_frac": by / (avg * 1e-3) / 1e9 / PEAK_HBM_GBS}


def deposit_roofline(r, pairs_per_deposit, fp32):
    """Shape-kernel source, the longer of its two node passes (normalisation,
    node sums), the other beside it: algorithmic flops of the (particle, node)
    pairs within R per launch over the pass's live HIP-event average.  The
    FP32 passes run on the matrix cores (peak FP32 MFMA), the FP64 ones on the
    vector units."""
    peak = PEAK_FP32_MFMA_TFLOPS if fp32 else PEAK_FP64_TFLOPS
    passes = []
    for cls, k32, k64, fpp in (("deposit_norm", "k_dep_norm_mfma", "k_dep_norm", DEP_FLOPS_NORM),
                               ("deposit_gather", "k_dep_gather_mfma", "k_dep_gather", DEP_FLOPS_GATHER)):
        n_launch, tot_ms = r["timing"][cls]
        if n_launch and pairs_per_deposit:
            avg = tot_ms / n_launch
            ach = pairs_per_deposit * fpp / (avg * 1e-3) / 1e12
            passes.append({"kernel": k32 if fp32 else k64, "avg_launch_ms": avg, "achieved": ach,
                           "frac": ach / peak, "flops_per_pair": fpp})
    if not passes:
        return None
    passes.sort(key=lambda q: -q["avg_launch_ms"])
    main = passes[0]
    out = {"bound": "mfma" if fp32 else "alu", "achieved": main["achieved"], "peak": peak, "unit": "TFLOP/s",
           "frac": main["frac"], "traffic": read_traffic(main["kernel"]) if fp32 else None,
           "kernel": main["kernel"], "avg_launch_ms": main["avg_launch_ms"],
           "pairs_within_R_per_launch": pairs_per_deposit, "flops_per_pair": main["flops_per_pair"]}
    if len(passes) > 1:
        other = dict(passes[1])
        other["traffic"] = read_traffic(other["kernel"]) if fp32 else None
        out["other_node_pass"] = other
    return out


# ---------------------------------------------------------------------------
# error against the oracle after the full step count
# ---------------------------------------------------------------------------
TRAPPED_HITS = 20   # particles pressed against a wall bounce this often or more in the oracle run


def error_statement(ro, rg, h):
    """Element and hit-count mismatch fractions and position errors (in element
    widths h) of the GPU run against the oracle.  Particles pressed against a
    curved wall by the field's normal component bounce off it every few stages,
    which amplifies rounding differences of any summation order; they are
    reported separately."""
    import numpy as np
    trapped = ro["hits"] >= TRAPPED_HITS
    same = (rg["elem"] == ro["elem"]) & (rg["status"] == ro["status"]) & (ro["status"] == 0)
    dx = np.linalg.norm(rg["x"] - ro["x"], axis=1) / h
    free = same & ~trapped
    return {"particles": int(len(ro["x"])), "elem_mismatch_frac": float((rg["elem"] != ro["elem"]).mean()),
            "status_mismatch": int((rg["status"] != ro["status"]).sum()),
            "free_hits_mismatch_frac": float((rg["hits"] != ro["hits"])[~trapped].mean()) if (~trapped).any() else 0.0,
            "free_max_err_h": float(dx[free].max(initial=0.0)),
            "free_rms_err_h": float(np.sqrt((dx[free] ** 2).mean())) if free.any() else 0.0,
            "wall_trapped": int(trapped.sum()),
            "trapped_hits_mismatch_frac": float((rg["hits"] != ro["hits"])[trapped].mean()) if trapped.any() else 0.0,
            "trapped_max_err_h": float(dx[same & trapped].max(initial=0.0))}


def oracle_run(w, idx, steps):
    import oracle as O
    o = O.Oracle(w.mesh, w.N, w.U)
    o.push(w.x[idx], w.v[idx], w.d[idx], w.elem_hint[idx])
    o.step(w.dt, steps, rk=w.rk, drag=w.drag)
    return o


def errors_vs_oracle(w, idx, steps, forms):
    """forms: name -> (U, precision, guess, weights); each GPU form runs the
    particle subset idx for `steps` steps and is compared with the oracle."""
    o = oracle_run(w, idx, steps)
    ro = o.read()
    out = {}
    for name, (U, prec, guess, wts) in forms.items():
        rg = run_gpu(w, U, prec, steps, 0, guess=guess, weights=wts, idx=idx)
        out[name] = error_statement(ro, rg["read"], w.mesh.h)
        out[name]["after_steps"] = steps
    return out, o


# ---------------------------------------------------------------------------
# learned guess
# ---------------------------------------------------------------------------
def train_guess(w, U, n_pairs, epochs, batch=1024, lr=2e-3, seed=4):
    """Newton-solved (features, xi) pairs from the first n_pairs particles, then
    fp_mlp_train on the GPU; returns weights and a training record."""
    import torch
    from paper_2211_05458_amd.lib import FlexiPart
    t0 = time.perf_counter()
    n = min(n_pairs, w.n_particles)
    g = FlexiPart(w.mesh, w.N, n)
    g.set_fluid_state(U)
    g.push(w.x[:n], w.v[:n], w.d[:n], w.elem_hint[:n])
    feat, xi = g.newton_pairs()
    wts, hist = g.mlp_train(feat, xi, epochs=epochs, batch=batch, lr=lr, seed=seed)
    torch.cuda.synchronize()
    pred = g.mlp_forward(wts, feat)
    med = float((pred - xi).abs().max(dim=1).values.median().item())
    g.close()
    return wts, {"pairs": int(feat.shape[0]), "epochs": epochs, "batch": batch, "seconds": time.perf_counter() - t0,
                 "loss_first_epoch": hist[0] if hist else None, "loss_last_epoch": hist[-1] if hist else None,
                 "median_guess_error": med}


def dep_list_rows(n_particles, n_elem, r):
    """Rows per element of the FP32 source's reuse list: a target stages about
    ppe (1 + 6 r + 3 pi r^2 + 4 pi r^3 / 3) particles (the element box grown by
    R = r h), with a quarter more room."""
    import math
    est = n_particles / n_elem * (1 + 6 * r + 3 * math.pi * r * r + 4 * math.pi * r ** 3 / 3)
    return int(math.ceil(1.25 * est / 64.0)) * 64


# ---------------------------------------------------------------------------
# the default line
# ---------------------------------------------------------------------------
def bench_composite(args):
    import numpy as np
    import torch
    from paper_2211_05458_amd import workloads as W
    import oracle as O
    K, Wm = args.steps, args.warmup
    log("generating the 96^3 two-way workload")
    t0 = time.perf_counter()
    w = W.config5(n_particles=args.particles or 20_000_000)
    log("generated in %.1f s" % (time.perf_counter() - t0))
    R = 1.5 * w.mesh.h
    per = np.array([1.0, 0.0, 1.0])
    S = {}

    rows = dep_list_rows(w.n_particles, w.mesh.n_elem, 1.5)

    def depositor(dtype):
        def dep(g):
            if "S" not in S or S["S"].dtype != dtype:
                S.clear()
                S["S"] = torch.zeros((g.E, 4, g.n3), dtype=dtype, device="cuda")
            if dtype == torch.float32 and getattr(g, "dep_list", None) is None:
                g.bind_deposit_list(rows)
            S["S"].zero_()
            g.deposit(S["S"], kind=1, radius=R, period=per)
        return dep

    U32 = torch.from_numpy(w.U.astype(np.float32)).cuda()
    log("learned guess: Newton pairs and training")
    wts, train = train_guess(w, U32, 1_000_000, args.epochs5)
    log("FP32 + learned-guess run")
    rv = run_gpu(w, U32, 1, K, Wm, guess=1, weights=wts, deposit=depositor(torch.float32), keep=True)
    g = rv.pop("ctx")
    V = g.node_volumes()
    tot_shape = (S["S"].double() * V[:, None, :]).sum(dim=(0, 2))
    Sn = g.deposit(None, kind=0, dtype=torch.float64)
    tot_near = (Sn * V[:, None, :]).sum(dim=(0, 2))
    cons = float(((tot_shape - tot_near).abs().max() / tot_near.abs().max()).item())
    del Sn, V
    # pairs within R of one more source from the final state (the timed
    # sources do not count them: counting costs the normalisation pass time)
    g.reset_stats()
    g.set_timing(False, count_pairs=True)
    depositor(torch.float32)(g)
    pairs = g.stats()["deposit_pairs"]
    g.set_timing(False)
    g.close()
    S.clear()
    value = summary(rv, K)
    value.update({"flagged_elements": rv["n_flagged"], "deposit_conservation_rel_err": cons,
                  "learned_guess": "enabled on the elements whose geometry deviates from the trilinear corner map "
                                   "by more than 0.05 h; %d of %d elements are that curved here"
                                   % (rv["n_flagged"], w.mesh.n_elem)})
    del U32
    torch.cuda.empty_cache()
    log("plain FP64 run")
    U64 = torch.from_numpy(w.U).cuda()
    r64 = run_gpu(w, U64, 0, K, Wm, deposit=depositor(torch.float64))
    S.clear()
    fp64 = summary(r64, K)
    fp64["roofline"] = deposit_roofline(r64, pairs, False)
    fp64["roofline_stage"] = stage_roofline(r64, w, K, 3)
    torch.cuda.empty_cache()
    log("error against the oracle (particle subset, %d steps)" % w.n_steps)
    idx = np.arange(0, w.n_particles, args.err_every)
    U32 = torch.from_numpy(w.U.astype(np.float32)).cuda()
    errs, o = errors_vs_oracle(w, idx, w.n_steps, {"fp32_learned": (U32, 1, 1, wts), "fp64": (U64, 0, 0, None)})
    # the FP32 source of the same subset after the full run (FP64 stepping, so
    # that only the source's arithmetic differs) against the oracle's source
    from paper_2211_05458_amd.lib import FlexiPart
    So = o.deposit(kind=1, radius=R, period=per)
    gs = FlexiPart(w.mesh, w.N, len(idx))
    gs.set_fluid_state(U64)
    gs.push(w.x[idx], w.v[idx], w.d[idx], w.elem_hint[idx])
    gs.step(w.dt, w.n_steps, rk=w.rk, drag=w.drag, precision=0)
    Sg = gs.deposit(None, kind=1, radius=R, period=per, dtype=torch.float32).cpu().numpy()
    src_err = float(np.abs(Sg - So).max() / np.abs(So).max())
    gs.close()
    del U32, U64
    torch.cuda.empty_cache()
    value["error_vs_oracle"] = errs["fp32_learned"]
    value["error_vs_oracle"]["fp32_source_max_rel_err"] = src_err
    fp64["error_vs_oracle"] = errs["fp64"]
    value["roofline_stage"] = stage_roofline(rv, w, K, 3, ubytes=4)
    roof = deposit_roofline(rv, pairs, True)

    cpu = None
    if not args.no_cpu_baseline:
        log("CPU oracle sample")
        cidx = np.arange(0, w.n_particles, args.cpu_every)
        oc = O.Oracle(w.mesh, w.N, w.U)
        oc.push(w.x[cidx], w.v[cidx], w.d[cidx], w.elem_hint[cidx])
        t0 = time.perf_counter()
        for _ in range(args.cpu_steps):
            oc.step(w.dt, 1, rk=w.rk, drag=w.drag)
            oc.deposit(kind=1, radius=R, period=per)
        el = time.perf_counter() - t0
        cpu = {"value": len(cidx) * args.cpu_steps / el, "unit": "particle-steps/s", "cores": O.num_threads(),
               "kind": "oracle", "cpu": cpu_model(),
               "sample": "one particle in %d (%d of %d) for %d steps of the same workload, each step followed by "
                         "the shape-kernel source, FP64, %.1f s wall (the oracle's step uses %d threads, its "
                         "source one)" % (args.cpu_every, len(cidx), w.n_particles, args.cpu_steps, el,
                                          O.num_threads())}
    del w
    annulus = None if args.no_annulus else bench_annulus_leg(args)
    out = {
        "metric": METRIC,
        "value": value["value"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": value["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "two-way coupling at scale: curved sine box 96^3 Ngeo=4, DG N=5 random-Fourier "
                               "state, %d particles, Schiller-Naumann, 3-stage LSERK, dt=1e-3, shape-kernel source "
                               "R=1.5h after every step; FP32 + learned-guess form" % rv["n_active"],
                   "elements": 884736, "particles": rv["n_active"], "N": 5, "n_geo": 4,
                   "newton_guess": ("continued reference coordinates of the previous stage first, then the "
                                    "learned guess on flagged elements, then the paper's guess (both forms)")
                   if WARM else "learned guess on flagged elements, then the paper's guess"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "fp32_learned": value,
        "fp64": fp64,
        "speedup_fp32_learned_vs_fp64": value["value"] / fp64["value"],
        "training": train,
        "annulus": annulus,
    }
    print(json.dumps(out))


def bench_annulus_leg(args):
    """Annular passage 48x24x48, Ngeo=6, N=5, 1e7 particles: plain FP64 against
    FP32 + learned guess (and the two halves of that change)."""
    import numpy as np
    import torch
    from paper_2211_05458_amd import workloads as W
    K, Wm = min(args.steps, args.annulus_steps), min(args.warmup, 2)
    log("generating the annulus workload")
    w = W.config4(n_particles=args.annulus_particles)
    U64 = torch.from_numpy(w.U).cuda()
    U32 = torch.from_numpy(w.U.astype(np.float32)).cuda()
    log("annulus: training")
    wts, train = train_guess(w, U64, 1_000_000, args.epochs)
    runs = {}
    for name, U, prec, guess in [("fp64", U64, 0, 0), ("fp64_learned", U64, 0, 1), ("fp32", U32, 1, 0),
                                 ("fp32_learned", U32, 1, 1)]:
        log("annulus run", name)
        runs[name] = run_gpu(w, U, prec, K, Wm, guess=guess, weights=wts if guess else None,
                             sort_every=ANNULUS_SORT)
    out = {"config": {"workload": "annular passage 48x24x48 Ngeo=6, DG N=5, %d particles, Schiller-Naumann, "
                                  "3-stage LSERK, dt=1e-3, sorted by element before every stage" % w.n_particles,
                      "elements": w.mesh.n_elem},
           "steps": K, "warmup": Wm, "training": train}
    for k, r in runs.items():
        out[k] = summary(r, K)
        out[k]["flagged_elements"] = r["n_flagged"]
        out[k]["roofline"] = stage_roofline(r, w, K, 3, ubytes=4 if k.startswith("fp32") else 8)
        km = r["kernel_ms"]
        out[k]["dominant_kernel"] = max(("stage_elem", "stage_lane", "track"), key=lambda c: km.get(c, 0.0))
    log("annulus: error against the oracle (particle subset, %d steps)" % w.n_steps)
    idx = np.arange(0, w.n_particles, args.err_every // 2)
    errs, _ = errors_vs_oracle(w, idx, w.n_steps, {"fp32_learned": (U32, 1, 1, wts), "fp64": (U64, 0, 0, None)})
    out["fp32_learned"]["error_vs_oracle"] = errs["fp32_learned"]
    out["fp64"]["error_vs_oracle"] = errs["fp64"]
    out["speedup_fp32_learned_vs_fp64"] = out["fp32_learned"]["value"] / out["fp64"]["value"]
    del U64, U32
    torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------------------
# other workloads (manual runs)
# ---------------------------------------------------------------------------
def pos_error(ref, other, h):
    """Position difference of two GPU runs from the same initial state."""
    import numpy as np
    both = (ref["read"]["status"] == 0) & (other["read"]["status"] == 0)
    dx = np.linalg.norm(other["read"]["x"][both] - ref["read"]["x"][both], axis=1)
    return {"pos_err_max_m": float(dx.max()), "pos_err_rms_m": float(np.sqrt((dx ** 2).mean())),
            "pos_err_max_h": float(dx.max() / h),
            "elem_mismatch_frac": float((other["read"]["elem"] != ref["read"]["elem"]).mean()),
            "hits_mismatch_frac": float((other["read"]["hits"] != ref["read"]["hits"]).mean())}


def bench_single(args):
    """One workload, FP64 and the alternative forms, per-kernel times."""
    import numpy as np
    import torch
    from paper_2211_05458_amd import workloads as W
    K, Wm = args.steps, args.warmup
    name = args.workload
    if name == "curved32":
        w = W.config2(n_particles=args.particles or 1_000_000)
    elif name == "precision":
        w = W.config3(n_particles=args.particles or 10_000_000)
    elif name == "annulus":
        w = W.config4(n_particles=args.particles or 10_000_000)
    elif name == "twoway":
        w = W.config5(n_particles=args.particles or 20_000_000)
    else:
        w = W.mortar_box(n_geo=4, N=5, refine=(2, 2), n_particles=args.particles or 1_000_000,
                         cells=(16, 16, 16), seed=1006)
    U64 = torch.from_numpy(w.U).cuda()
    U32 = torch.from_numpy(w.U.astype(np.float32)).cuda()
    dep = None
    if name == "twoway":
        R, per, S = 1.5 * w.mesh.h, np.array([1.0, 0.0, 1.0]), {}

        rows = dep_list_rows(w.n_particles, w.mesh.n_elem, 1.5)

        def dep(g):
            if "S" not in S:
                S["S"] = torch.zeros((g.E, 4, g.n3), dtype=torch.float32, device="cuda")
            if getattr(g, "dep_list", None) is None:
                g.bind_deposit_list(rows)
            S["S"].zero_()
            g.deposit(S["S"], kind=1, radius=R, period=per)
    sort_every = args.sort_every if args.sort_every is not None else (ANNULUS_SORT if name == "annulus" else 1)
    forms = [("fp64", U64, 0, 0)] if name != "twoway" else []
    forms += [("fp32", U32, 1, 0)]
    if name == "mortar":
        forms = [("fp64", U64, 0, 0), ("fp64_refspace", U64, 0, 0)]
    runs = {}
    for fname, U, prec, guess in forms:
        log("run", fname)
        runs[fname] = run_gpu(w, U, prec, K, Wm, guess=guess, deposit=dep,
                              tracking=1 if fname.endswith("refspace") else 0, sort_every=sort_every)
    out = {"metric": METRIC, "workload": name, "steps": K, "warmup": Wm, "particles": w.n_particles,
           "elements": w.mesh.n_elem}
    first = None
    for k, r in runs.items():
        out[k] = summary(r, K)
        out[k]["roofline"] = stage_roofline(r, w, K, 3 if w.rk == 1 else 5, ubytes=4 if k.startswith("fp32") else 8)
        out[k]["stats"] = r["stats"]
        if first is None:
            first = r
        else:
            out[k].update(pos_error(first, r, w.mesh.h))
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
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--particles", type=int, default=None)
    ap.add_argument("--workload", choices=["default", "curved32", "annulus", "precision", "twoway", "mortar"],
                    default="default", help="default: the benchmark line; the others measure one workload")
    ap.add_argument("--epochs", type=int, default=20, help="learned-guess training epochs (annulus leg)")
    ap.add_argument("--epochs5", type=int, default=3, help="learned-guess training epochs (two-way workload)")
    ap.add_argument("--annulus-particles", type=int, default=10_000_000)
    ap.add_argument("--annulus-steps", type=int, default=10, help="timed steps of the annulus leg")
    ap.add_argument("--no-annulus", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--err-every", type=int, default=10000, help="error subset: every k-th particle")
    ap.add_argument("--cpu-every", type=int, default=2500, help="oracle sample: every k-th particle")
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--sort-every", type=int, default=None,
                    help="--workload runs: sort by element every k steps (negative: before every stage); "
                         "default: before every stage on the annular passage, every step elsewhere")
    ap.add_argument("--no-warm", action="store_true",
                    help="locate with the paper's initial guess only (no continued reference coordinates)")
    ap.add_argument("--mode", choices=["bench", "copy"], default="bench",
                    help="copy: a plain device copy of known size, the calibration for HBM counters")
    args = ap.parse_args()
    global WARM
    WARM = 0 if args.no_warm else 2
    if args.mode == "copy":
        copy_calibration()
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    from paper_2211_05458_amd import workloads as W
    W.VERBOSE = True
    if args.workload == "default":
        bench_composite(args)
    else:
        bench_single(args)


if __name__ == "__main__":
    main()
