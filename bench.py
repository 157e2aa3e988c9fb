#!/usr/bin/env python3
"""Throughput of the spin/polarisation-resolved SF-QED particle step on one MI355X.

Workload (the focused-pulse configuration): 1e7 electrons, gamma0 = 2000 (10 % spread),
1 mrad divergence, unpolarised, colliding head-on with a circularly polarised focused
pulse (w0 = 3 um, a0 = 100, 10 cycles), dt = T0/500, NCS with spin flip and photon Stokes
output.  The bunch is placed at the collision (step 2400 of the 6000-step run) so the
timed steps see the peak field.  One step = one fused gather + Boris + T-BMT + NCS pass
over all electrons, with photons appended in order.

Prints one JSON line: mixed-precision particle-steps/s (the headline), the FP64 GPU path
on the same input and draws, their spectrum / spin / polarisation differences, the
roofline of the fused kernel and the CPU oracle on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic bytes per lepton-step (every lepton, the decide kernel): read x, p (48 B),
# S, id (8 B); write x, p (48 B), S.  S is 3 x 4 B (mixed) or 3 x 8 B (FP64).
BYTES_LEPTON = {"mixed": 48 + 12 + 8 + 48 + 12, "fp64": 48 + 24 + 8 + 48 + 24}
# per emitted photon (the event kernel): read the parent weight (8 B); write x, k, w
# (56 B), xi and e1 (6 x 4 or 6 x 8 B), id (8 B), alive (1 B)
BYTES_PHOTON = {"mixed": 8 + 56 + 24 + 8 + 1, "fp64": 8 + 56 + 48 + 8 + 1}
KERNEL_SOURCES = ["qed_kernels.hip", "qed_dev.hpp", "qed_internal.hpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_lepton_decide_c2.json")
# one benchmark step = one qed_step_leptons call = three launches on the stream: decide
# (all leptons), scan (event counts), events (emitting leptons).  HIP events bracket each
# call and, through qed_set_step_events, each launch.


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2306_11288_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(prec: str):
    """HBM bytes per decide launch from the committed counter summary, if it was taken on
    the current kernel sources; else None."""
    try:
        d = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if d.get("kernel_hash") != kernel_hash():
        return None
    return d.get(prec, {}).get("bytes_per_launch")


EV_EVERY = 10   # timed steps per step with per-launch events


def run_gpu(prec, cfg, steps, warmup, torch, Q, per_launch_events=True, learned=False, photon_cap=None):
    precision = Q.QED_MIXED if prec == "mixed" else Q.QED_FP64
    n = len(cfg["leptons"]["x"])
    ctx = Q.Context(dt=cfg["dt"], procs=cfg["procs"], seed=cfg["seed"], id_start=cfg["next_id"],
                    precision=precision)
    if learned:
        ctx.mlp_load_pretrained()
        ctx.set_sampler(Q.SAMPLER_MLP)
    L = Q.Leptons.from_state(cfg["leptons"], precision=precision)
    cap = photon_cap or int(n * 0.03 * (steps + warmup)) + 1_000_000
    G = Q.Photons(cap, precision=precision)
    segs = Q.whole(cfg["field"])
    s0 = cfg["start_step"]
    tuning = ctx.autotune(segs, L, s0, reps=3)
    for s in range(s0, s0 + warmup):
        ctx.step_leptons(segs, L, G, s)
    torch.cuda.synchronize()
    n_before = G.count
    stream = torch.cuda.current_stream()
    # every EV_EVERY-th timed step: four events recorded by the library around its launches
    # (each event record is a barrier that costs the device a few microseconds, so the
    # steps between the sampled ones run uninstrumented, as in production)
    sampled = [k for k in range(steps) if k % EV_EVERY == 0] if per_launch_events else []
    ev = {k: [torch.cuda.Event(enable_timing=True) for _ in range(4)] for k in sampled}
    for e4 in ev.values():   # create the HIP events before the timed region
        for e in e4:
            e.record(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k, s in enumerate(range(s0 + warmup, s0 + warmup + steps)):
        if per_launch_events:
            ctx.set_step_events(ev.get(k))
        ctx.step_leptons(segs, L, G, s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.set_step_events(None)
    ev = [ev[k] for k in sampled]
    kern = {}
    if per_launch_events:
        kern = {"step": [e[0].elapsed_time(e[3]) for e in ev], "decide": [e[0].elapsed_time(e[1]) for e in ev],
                "scan": [e[1].elapsed_time(e[2]) for e in ev], "events": [e[2].elapsed_time(e[3]) for e in ev]}
    status = ctx.read_status()
    return {"ctx": ctx, "L": L, "G": G, "wall": wall, "kern_ms": kern, "n": n, "tuning": tuning,
            "photons_timed": G.count - n_before, "photons_total": G.count, "photon_start": n_before,
            "status": status}


def copy_bandwidth(torch, mib=2048, reps=5):
    """Achievable HBM bandwidth of a plain elementwise copy (x * 1.0, float64): bytes read +
    written per second, best of `reps`."""
    src = torch.ones((mib << 20) // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    best = float("inf")
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        torch.mul(src, 1.0, out=dst)
        b.record()
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b))
    del src, dst
    return 2 * (mib << 20) / (best * 1e-3) / 1e9


def detector_stokes(G, start, torch):
    """Stokes vectors of photons [start, count) rotated to the detector basis (y, z)
    projected transverse to each photon's direction (the post-processing step of
    Algorithm 1)."""
    n = G.count
    sl = slice(start, n)
    k = torch.stack([G.kx[sl], G.ky[sl], G.kz[sl]]).double()
    nh = k / torch.linalg.norm(k, dim=0)
    e1 = torch.stack([G.e1x[sl], G.e1y[sl], G.e1z[sl]]).double()
    yh = torch.zeros_like(nh)
    yh[1] = 1.0
    d1 = yh - nh * (yh * nh).sum(0)
    d1 = d1 / torch.linalg.norm(d1, dim=0)
    e2 = torch.cross(nh, e1, dim=0)
    c, s = (e1 * d1).sum(0), (e2 * d1).sum(0)
    c2, s2 = c * c - s * s, 2 * c * s
    x1, x2, x3 = G.xi1[sl].double(), G.xi2[sl].double(), G.xi3[sl].double()
    return torch.stack([c2 * x1 - s2 * x3, x2, s2 * x1 + c2 * x3])


def error_metrics(a, b, gamma0, torch):
    """Mixed (b) against FP64 (a) after the same steps from the same state and draws."""
    out = {}
    La, Lb = a["L"], b["L"]
    n = a["n"]
    ea = torch.sqrt(1 + La.px[:n] ** 2 + La.py[:n] ** 2 + La.pz[:n] ** 2)
    eb = torch.sqrt(1 + Lb.px[:n] ** 2 + Lb.py[:n] ** 2 + Lb.pz[:n] ** 2)
    out["mean_energy_rel"] = abs(float(eb.mean() / ea.mean()) - 1)

    def hist(x, lo, hi, bins, log=False):
        x = x.double()
        if log:
            x = torch.log10(x.clamp_min(1e-300))
        h = torch.histc(x.float(), bins=bins, min=lo, max=hi).double()
        return h / max(float(h.sum()), 1.0)

    def l1(h1, h2):
        return float((h1 - h2).abs().sum())

    Ga, Gb = a["G"], b["G"]
    sa, sb = a["photon_start"], b["photon_start"]
    wa = torch.sqrt(Ga.kx[sa:Ga.count] ** 2 + Ga.ky[sa:Ga.count] ** 2 + Ga.kz[sa:Ga.count] ** 2) / gamma0
    wb = torch.sqrt(Gb.kx[sb:Gb.count] ** 2 + Gb.ky[sb:Gb.count] ** 2 + Gb.kz[sb:Gb.count] ** 2) / gamma0
    out["photon_spectrum_L1"] = l1(hist(wa, -5, 0, 100, True), hist(wb, -5, 0, 100, True))
    out["photon_count_rel"] = abs((Gb.count - sb) / max(Ga.count - sa, 1) - 1)
    for name, (ta, tb) in {"electron_theta_y_L1": (La.py[:n] / La.px[:n], Lb.py[:n] / Lb.px[:n]),
                           "electron_theta_z_L1": (La.pz[:n] / La.px[:n], Lb.pz[:n] / Lb.px[:n]),
                           "photon_theta_y_L1": (Ga.ky[sa:Ga.count] / Ga.kx[sa:Ga.count],
                                                 Gb.ky[sb:Gb.count] / Gb.kx[sb:Gb.count])}.items():
        out[name] = l1(hist(ta, -0.05, 0.05, 100), hist(tb, -0.05, 0.05, 100))
    Sa = torch.stack([La.sx[:n], La.sy[:n], La.sz[:n]]).double().mean(1)
    Sb = torch.stack([Lb.sx[:n], Lb.sy[:n], Lb.sz[:n]]).double().mean(1)
    out["mean_spin_abs_diff"] = float(torch.linalg.norm(Sa - Sb))
    out["polarisation_degree_fp64"] = float(torch.linalg.norm(Sa))
    out["polarisation_degree_mixed"] = float(torch.linalg.norm(Sb))
    xa, xb = detector_stokes(Ga, sa, torch).mean(1), detector_stokes(Gb, sb, torch).mean(1)
    out["photon_xi2_abs_diff"] = abs(float(xa[1] - xb[1]))
    out["photon_xi3_abs_diff"] = abs(float(xa[2] - xb[2]))
    out["photon_xi3_detector_fp64"] = float(xa[2])
    return out


# metrics that measure a difference between two runs (the others are values)
DIFF_METRICS = ("mean_energy_rel", "photon_spectrum_L1", "photon_count_rel", "electron_theta_y_L1",
                "electron_theta_z_L1", "photon_theta_y_L1", "mean_spin_abs_diff", "photon_xi2_abs_diff",
                "photon_xi3_abs_diff")


def tolerance_check(err: dict, stat: dict) -> dict:
    """Each difference metric against max(4 x its value between two FP64 runs with different
    random draws, 1e-3): the accuracy bar the mixed (or learned) run is stated at."""
    tol = {k: max(4.0 * stat[k], 1e-3) for k in DIFF_METRICS}
    return {"tolerance": tol, "within": {k: err[k] <= tol[k] for k in DIFF_METRICS},
            "all_within": all(err[k] <= tol[k] for k in DIFF_METRICS)}


class _Cat:
    """Concatenated view of several lepton lists (for the error metrics)."""

    def __init__(self, lists, torch):
        for k in ("x", "y", "z", "px", "py", "pz", "sx", "sy", "sz"):
            setattr(self, k, torch.cat([getattr(L, k)[:L.count] for L in lists]))


def run_batched(args, torch, Q, W):
    """Many collisions (64, log-uniform 1e3..2e6 electrons, own laser each) in one list:
    autotuned launch shape, K steps captured in a hipGraph with a device step counter and
    replayed, in both precisions; against the same collisions stepped one at a time (eager,
    FP64).  The batching gain is batched FP64 over one-by-one FP64 (same arithmetic); the
    precision gain is batched mixed over batched FP64."""
    start = 100
    cfg = W.c4(start_step=start)
    n = len(cfg["leptons"]["x"])
    K = 10
    reps = max(1, args.batch_steps // K)
    steps = K * reps
    cap = int(n * 0.04 * (steps + 2)) + 100_000
    segs = Q.segments(cfg["segments"])

    def batched(precision):
        ctx = Q.Context(dt=cfg["dt"], procs=cfg["procs"], seed=cfg["seed"], id_start=cfg["next_id"],
                        precision=precision)
        L = Q.Leptons.from_state(cfg["leptons"], precision=precision)
        G = Q.Photons(cap, precision=precision)
        tuning = ctx.autotune(segs, L, start, reps=2)
        ctx.step_leptons(segs, L, G, start)   # eager step: staging sized, segments uploaded
        counter = torch.zeros(1, dtype=torch.int64, device="cuda")
        torch.cuda.synchronize()
        ctx.set_step_counter(counter)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for _ in range(K):
                ctx.step_leptons(segs, L, G, start + 1)
                ctx.advance_step(1)
        torch.cuda.synchronize()
        n0 = G.count
        t0 = time.perf_counter()
        for _ in range(reps):
            g.replay()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ctx.set_step_counter(None)
        return {"wall": wall, "L": L, "G": G, "n0": n0, "status": ctx.read_status(), "tuning": tuning}

    bm = batched(Q.QED_MIXED)
    bd = batched(Q.QED_FP64)
    # one collision at a time, FP64, eager
    ctx64 = Q.Context(dt=cfg["dt"], procs=cfg["procs"], seed=cfg["seed"], id_start=cfg["next_id"], precision=Q.QED_FP64)
    lists, fsegs = [], []
    for (b, e, spec) in cfg["segments"]:
        lists.append(Q.Leptons.from_state({k: v[b:e] for k, v in cfg["leptons"].items()}, precision=Q.QED_FP64))
        fsegs.append(Q.whole(spec))
    G64 = Q.Photons(cap, precision=Q.QED_FP64)
    for Lk, sk in zip(lists, fsegs):
        ctx64.step_leptons(sk, Lk, G64, start)
    torch.cuda.synchronize()
    m0 = G64.count
    t0 = time.perf_counter()
    for s in range(start + 1, start + 1 + steps):
        for Lk, sk in zip(lists, fsegs):
            ctx64.step_leptons(sk, Lk, G64, s)
    torch.cuda.synchronize()
    wall_1 = time.perf_counter() - t0
    one = {"L": _Cat(lists, torch), "G": G64, "n": n, "photon_start": m0}

    def view(r):
        return {"L": r["L"], "G": r["G"], "n": n, "photon_start": r["n0"]}

    def line(r, bytes_per):
        v = n * steps / r["wall"]
        return {"value": v, "ms_per_step": 1e3 * r["wall"] / steps, "status_bits": r["status"],
                "tuning": r["tuning"], "hbm_frac": v * bytes_per / (HBM_PEAK_GBS * 1e9)}
    return {"workload": f"{len(cfg['sizes'])} collisions, {n} electrons (log-uniform 1e3..2e6 each), plane-wave "
                        f"sin^2 8-cycle lasers, a0 U(10,200), gamma0 U(500,5000), LP/CP; dt = T0/400, steps "
                        f"{start + 1}..{start + steps}",
            "electrons": n, "steps": steps, "graph_steps_per_replay": K,
            "batched_graph_mixed": line(bm, BYTES_LEPTON["mixed"]),
            "batched_graph_fp64": line(bd, BYTES_LEPTON["fp64"]),
            "one_by_one_fp64": {"value": n * steps / wall_1, "ms_per_step": 1e3 * wall_1 / steps,
                                "launches_per_step": 3 * len(lists)},
            "batching_gain_fp64": wall_1 / bd["wall"],
            "precision_gain_batched": bd["wall"] / bm["wall"],
            "error_batched_fp64_vs_one_by_one": error_metrics(one, view(bd), 5000.0, torch),
            "error_batched_mixed_vs_one_by_one_fp64": error_metrics(one, view(bm), 5000.0, torch),
            "photons_per_step": (bm["G"].count - bm["n0"]) / steps}


MLP_FLOP = 2 * (4 * 128 + 2 * 128 * 128 + 128 * 3)   # multiply-adds x 2 per sample (forward)
MFMA_BF16_PEAK_TFLOPS = 2500.0
# training, matrix-core work per sample: the two 128 x 128 layers forward, backward through
# the activations, and their weight gradients (the VALU layers 1 and 4 not counted)
MLP_TRAIN_MFMA_FLOP = 3 * 2 * (2 * 128 * 128)
MFMA_FP32_PEAK_TFLOPS = 157.3


def run_learned(args, torch, Q, W, cfg, fp64, fp64_b=None):
    """The learned sampler: matrix-core inference against the table sampler on the same
    inputs, training throughput of the library's kernels, and the focused-pulse step with
    the network (the shipped one) as sampler against the FP64 table path."""
    from paper_2306_11288_amd.train_sampler import train
    out = {}
    ctx = Q.Context(dt=cfg["dt"], procs=cfg["procs"], seed=cfg["seed"], id_start=cfg["next_id"],
                    precision=Q.QED_MIXED)
    ctx.mlp_load_pretrained()
    n = 1 << 23
    X, T64 = ctx.mlp_samples(n, seed=77)
    Y = torch.empty((n, 3), dtype=torch.float32, device="cuda")

    def best_ms(fn, reps=5):
        b = float("inf")
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            b = min(b, e0.elapsed_time(e1))
        return b
    t_mlp = best_ms(lambda: ctx.mlp_forward(X, Y))
    err_mlp = (Y - T64).abs().mean(0).cpu().tolist()
    t_tab = best_ms(lambda: ctx.sampler_table(X, Y))
    err_tab = (Y - T64).abs().mean(0).cpu().tolist()
    tflops = MLP_FLOP * n / (t_mlp * 1e-3) / 1e12
    out["sampler"] = {
        "samples": n, "network_samples_per_s": n / (t_mlp * 1e-3), "table_samples_per_s": n / (t_tab * 1e-3),
        "network_mean_abs_error_vs_fp64_table": err_mlp, "fp32_table_mean_abs_error_vs_fp64_table": err_tab,
        "network_bytes_bf16": Q.MLP_NPARAM * 2, "table_bytes_fp32": 4 * 2 * 512 * 1024,
        "roofline": {"bound": "mfma", "achieved": tflops, "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": tflops / MFMA_BF16_PEAK_TFLOPS, "kernel": "k_mlp_forward (bf16 MFMA 32x32x16)",
                     "flop_per_sample": MLP_FLOP, "avg_launch_ms": t_mlp},
        # the vector-unit work the matrix cores cannot take: layer 1 (512 FMA), layer 4
        # (384), per SiLU 3 full-rate ops + v_exp and v_rcp at a quarter rate (384 SiLU)
        "roofline_alu": {"bound": "alu", "achieved": n / (t_mlp * 1e-3) * MLP_VALU_OPS / 1e12,
                         "peak": VALU_LANE_OPS_PEAK / 1e12, "unit": "Tlane-op/s",
                         "frac": n / (t_mlp * 1e-3) * MLP_VALU_OPS / VALU_LANE_OPS_PEAK,
                         "lane_ops_per_sample": MLP_VALU_OPS,
                         "peak_note": "256 CUs x 64 lanes x 2.4 GHz, one FP32 (non-packed) op per lane per clock; "
                                      "a transcendental counts 4"},
    }
    del X, T64, Y
    out["nbw"] = run_learned_nbw(torch, Q, W, best_ms)
    c2 = Q.Context(dt=0.01, procs=Q.PROC_NCS | Q.PROC_NCS_STOKES, seed=1, id_start=0, precision=Q.QED_MIXED)
    # the training step alone (three launches: forward + backward through the activations,
    # weight gradients, ordered sum + Adam), pairs resident, at the trainer's batch and at
    # a batch that fills the chip
    c2.mlp_init(seed=4)
    Xt, Tt = c2.mlp_samples(1 << 20, seed=6)
    lossb = torch.empty(1, dtype=torch.float32, device="cuda")
    steps_out = {}
    for B in (8192, 65536):
        reps = 20

        def run_steps():
            for k in range(reps):
                j = (k * B) % (Xt.shape[0] - B + 1)
                c2.mlp_train_step(Xt[j:j + B], Tt[j:j + B], 1e-5, (1.0, 0.3, 0.3), lossb)
        run_steps()
        ms = best_ms(run_steps, reps=3) / reps
        tf = MLP_TRAIN_MFMA_FLOP * B / (ms * 1e-3) / 1e12
        steps_out[str(B)] = {"us_per_step": 1e3 * ms, "samples_per_s": B / (ms * 1e-3),
                             "roofline": {"bound": "mfma", "achieved": tf, "peak": MFMA_FP32_PEAK_TFLOPS,
                                          "unit": "TFLOP/s", "frac": tf / MFMA_FP32_PEAK_TFLOPS,
                                          "flop_per_sample": MLP_TRAIN_MFMA_FLOP,
                                          "kernels": "k_train_fb + k_train_dw (FP32 MFMA 32x32x2) + k_train_reduce"}}
    out["training_step"] = steps_out
    del Xt, Tt
    tr = train(c2, n_samples=args.train_samples, epochs=1.0, batch=8192, seed=5)
    out["training"] = {"samples": tr["samples"], "steps": tr["steps"], "batch": tr["batch"], "seconds": tr["seconds"],
                       "samples_per_s": tr["samples"] / tr["seconds"], "val_mae_after": tr["val_after"]["mae"],
                       "note": "one epoch from fresh weights, timing includes generating the pairs"}
    learned = run_gpu("mixed", cfg, args.steps, args.warmup, torch, Q, per_launch_events=False, learned=True)
    out["step"] = {"value": args.n * args.steps / learned["wall"], "ms_per_step": 1e3 * learned["wall"] / args.steps,
                   "status_bits": learned["status"], "network": "sampler_ncs.npy (5e7 pairs, 2 epochs)"}
    if fp64 is not None:
        out["step"]["error_vs_fp64"] = error_metrics(fp64, learned, 2000.0, torch)
        if fp64_b is not None:
            out["step"]["error_tolerance"] = tolerance_check(out["step"]["error_vs_fp64"],
                                                             error_metrics(fp64, fp64_b, 2000.0, torch))
    return out


def run_learned_nbw(torch, Q, W, best_ms) -> dict:
    """The NBW network (the shipped one): inference against the NBW table sampler on the
    same inputs, and the pair step with the network against the table on the same photons
    and draws (plane wave a0 = 300 at its peak, 2e6 photons of 1.5 GeV, mixed precision)."""
    import numpy as np
    out = {}
    ctx = Q.Context(dt=0.01, procs=Q.PROC_NBW, seed=1, id_start=0, precision=Q.QED_MIXED)
    ctx.mlp_load_pretrained(net=Q.NET_NBW)
    n = 1 << 23
    X, T64 = ctx.mlp_samples(n, seed=78)
    Y = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    t_mlp = best_ms(lambda: ctx.mlp_forward(X, Y))
    err_mlp = (Y - T64).abs().mean(0).cpu().tolist()
    t_tab = best_ms(lambda: ctx.sampler_table(X, Y))
    err_tab = (Y - T64).abs().mean(0).cpu().tolist()
    out["sampler"] = {"samples": n, "network_samples_per_s": n / (t_mlp * 1e-3),
                      "table_samples_per_s": n / (t_tab * 1e-3),
                      "network_mean_abs_error_vs_fp64_table": err_mlp,
                      "fp32_table_mean_abs_error_vs_fp64_table": err_tab,
                      "network_bytes_bf16": Q.MLP_NPARAM * 2, "table_bytes_fp32": 4 * 2 * 256 * 512,
                      "outputs": "delta, mean positron / electron spin along b"}
    del X, T64, Y
    npho, steps, s0 = 2_000_000, 20, 2000
    st = W.photons(npho, seed=45, eps0=3000.0, eps_rel_spread=0.2, divergence=2e-3, x_mean=-2.0, x_sigma=1.0,
                   r_sigma=1.0, id0=0)
    spec = {"kind": W.FIELD_PW, "circular": 0, "a0": 300.0, "ncycles": 8.0, "phase0": 0.3, "pol_angle": 0.4,
            "phi_start": 0.0}
    k = torch.as_tensor(np.sqrt(st["kx"] ** 2 + st["ky"] ** 2 + st["kz"] ** 2), device="cuda")
    res = {}
    for name, sampler in (("table", Q.SAMPLER_TABLE), ("network", Q.SAMPLER_MLP_NBW)):
        c = Q.Context(dt=W.TWO_PI / 500, procs=Q.PROC_VB | Q.PROC_NBW, seed=9, id_start=1 << 41,
                      precision=Q.QED_MIXED)
        c.mlp_load_pretrained(net=Q.NET_NBW)
        c.set_sampler(sampler)
        G = Q.Photons.from_state(st, precision=Q.QED_MIXED)
        em, ep = Q.Leptons(400_000, -1, precision=Q.QED_MIXED), Q.Leptons(400_000, 1, precision=Q.QED_MIXED)
        segs = Q.whole(spec)
        c.step_photons(segs, G, em, ep, s0)          # warm-up (first launch of each kernel)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(s0 + 1, s0 + 1 + steps):
            c.step_photons(segs, G, em, ep, s)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        res[name] = {"ms_per_step": 1e3 * wall / steps, "pairs": int(ep.count), "status_bits": c.read_status(),
                     "ep": ep, "alive": G.alive[:npho].clone()}
    same_pairs = (res["table"]["pairs"] == res["network"]["pairs"] and
                  bool(torch.equal(res["table"]["alive"], res["network"]["alive"])))
    # the same photons convert in both runs and the pairs come in the same order, so the
    # positron energies compare pair by pair and as spectra
    dead = torch.nonzero(res["table"]["alive"] == 0).flatten()
    step_err = None
    if same_pairs:
        en = {}
        for name in ("table", "network"):
            ep = res[name]["ep"]
            m = ep.count
            en[name] = torch.sqrt(1 + ep.px[:m].double() ** 2 + ep.py[:m].double() ** 2 + ep.pz[:m].double() ** 2)
        scale = en["table"].mean()
        ht = torch.histc(en["table"] / scale, bins=40, min=0, max=4)
        hn = torch.histc(en["network"] / scale, bins=40, min=0, max=4)
        step_err = {"positron_energy_hist_L1": float((ht - hn).abs().sum() / ht.sum()),
                    "positron_mean_energy_rel": float((en["network"].mean() / scale - 1).abs()),
                    "positron_energy_mean_abs_rel_diff": float(((en["network"] - en["table"]) / en["table"]).abs().mean())}
    out["pair_step"] = {"photons": npho, "steps": steps, "start_step": s0, "converted": int(dead.numel()),
                        "pairs_per_step": res["table"]["pairs"] / (steps + 1),
                        "ms_per_step_table": res["table"]["ms_per_step"],
                        "ms_per_step_network": res["network"]["ms_per_step"],
                        "same_decisions": same_pairs, "error_vs_table": step_err,
                        "status_bits": [res["table"]["status_bits"], res["network"]["status_bits"]],
                        "what": "photon VB + NBW step, plane wave a0 = 300 near its peak, mixed precision"}
    return out


def run_full_interaction(args, torch, Q, W) -> dict:
    """The whole focused-pulse interaction (the workload's 6000 steps, from before the bunch
    meets the pulse until after it has left) on a bunch of fewer electrons, in mixed
    precision, in FP64 and in FP64 with other random draws: the mixed result's error after
    the full interaction, against the statistical spread of two FP64 runs."""
    n, steps = args.full_n, args.full_steps
    cfg = W.c2(n, start_step=0)
    runs = {}
    for name, prec, c in (("mixed", "mixed", cfg), ("fp64", "fp64", cfg),
                          ("fp64_b", "fp64", dict(cfg, seed=cfg["seed"] + 1))):
        runs[name] = run_gpu(prec, c, steps, 0, torch, Q, per_launch_events=False, photon_cap=40 * n)
    err = error_metrics(runs["fp64"], runs["mixed"], 2000.0, torch)
    stat = error_metrics(runs["fp64"], runs["fp64_b"], 2000.0, torch)
    out = {"workload": f"{n} electrons of the focused-pulse recipe, steps 0..{steps - 1} (the whole interaction)",
           "photons_per_electron": {k: runs[k]["G"].count / n for k in runs},
           "mixed_particle_steps_per_s": n * steps / runs["mixed"]["wall"],
           "fp64_particle_steps_per_s": n * steps / runs["fp64"]["wall"],
           "status_bits": {k: runs[k]["status"] for k in runs},
           "error_vs_fp64": err, "error_statistical_fp64_seeds": stat,
           "error_tolerance": tolerance_check(err, stat)}
    for k in list(runs):
        runs[k]["ctx"].close()
    del runs
    torch.cuda.empty_cache()
    return out


# vector work of one forward sample in full-rate lane operations: layers 1 and 4 (FMA),
# and per SiLU 3 ops plus two transcendentals at a quarter of the rate
MLP_VALU_OPS = 4 * 128 + 128 * 3 + 3 * 128 * (3 + 2 * 4)
VALU_LANE_OPS_PEAK = 256 * 64 * 2.4e9

# Yee step: three passes, each reading 6 components and writing 3 (FP32)
BYTES_YEE_NODE = 3 * (6 + 3) * 4
# current deposition per lepton: read the start and end positions and the weight (FP64); the
# atomics land in the 12.6 MB current grid, which stays in the caches
BYTES_DEPOSIT = 7 * 8
# charge of a unit-weight macro-particle in the field equations' units for the cascade: the
# beam's own field stays far below the laser's (the cost does not depend on it)
CASCADE_QSCALE = 1e-4
# photon step: read x, k, xi, e1, id, alive; write x, xi, e1
BYTES_PHOTON_STEP = {"mixed": 24 + 24 + 12 + 12 + 8 + 1 + 24 + 12 + 12, "fp64": 24 + 24 + 24 + 24 + 8 + 1 + 24 + 24 + 24}


def cascade_summary(em, ep, G, gamma0, torch):
    """Histograms and means of one cascade run's final lists (for the error metrics)."""
    def hist(x, lo, hi, bins):
        h = torch.histc(x.float(), bins=bins, min=lo, max=hi).double()
        return h / max(float(h.sum()), 1.0)

    out = {}
    for name, L in (("electron", em), ("positron", ep)):
        n = L.count
        p = torch.stack([L.px[:n], L.py[:n], L.pz[:n]]).double()
        e = torch.sqrt(1 + (p * p).sum(0))
        out[name + "_count"] = n
        out[name + "_mean_energy"] = float(e.mean()) if n else 0.0
        out[name + "_mean_spin"] = (torch.stack([L.sx[:n], L.sy[:n], L.sz[:n]]).double().mean(1).cpu()
                                    if n else torch.zeros(3, dtype=torch.float64))
        out[name + "_theta_y"] = hist(torch.atan2(p[1], p[0]), -math.pi, math.pi, 200)
    n = G.count
    k = torch.stack([G.kx[:n], G.ky[:n], G.kz[:n]]).double()
    w = torch.sqrt((k * k).sum(0))
    out["photon_count"] = n
    out["photon_spectrum"] = hist(torch.log10((w / gamma0).clamp_min(1e-300)), -5.0, 0.0, 100)
    out["photon_theta_y"] = hist(torch.atan2(k[1], k[0]), -math.pi, math.pi, 200)
    out["photon_xi_detector"] = detector_stokes(G, 0, torch).mean(1).cpu()
    out["photons_alive"] = int(G.alive[:n].sum())
    return out


# difference metrics of the cascade (mixed against FP64, or FP64 between two seeds)
CASCADE_DIFF = ("electron_mean_energy_rel", "positron_count_rel", "positron_mean_energy_rel", "photon_count_rel",
                "photon_spectrum_L1", "electron_theta_y_L1", "photon_theta_y_L1", "electron_mean_spin_abs_diff",
                "positron_mean_spin_abs_diff", "photon_xi2_abs_diff", "photon_xi3_abs_diff")


def cascade_metrics(a, b):
    rel = lambda x, y: abs(x / y - 1) if y else abs(x - y)
    l1 = lambda h1, h2: float((h1 - h2).abs().sum())
    return {"electron_mean_energy_rel": rel(b["electron_mean_energy"], a["electron_mean_energy"]),
            "positron_count_rel": rel(b["positron_count"], a["positron_count"]),
            "positron_mean_energy_rel": rel(b["positron_mean_energy"], a["positron_mean_energy"]),
            "photon_count_rel": rel(b["photon_count"], a["photon_count"]),
            "photon_spectrum_L1": l1(a["photon_spectrum"], b["photon_spectrum"]),
            "electron_theta_y_L1": l1(a["electron_theta_y"], b["electron_theta_y"]),
            "photon_theta_y_L1": l1(a["photon_theta_y"], b["photon_theta_y"]),
            "electron_mean_spin_abs_diff": float((a["electron_mean_spin"] - b["electron_mean_spin"]).norm()),
            "positron_mean_spin_abs_diff": float((a["positron_mean_spin"] - b["positron_mean_spin"]).norm()),
            "photon_xi2_abs_diff": abs(float(a["photon_xi_detector"][1] - b["photon_xi_detector"][1])),
            "photon_xi3_abs_diff": abs(float(a["photon_xi_detector"][2] - b["photon_xi_detector"][2]))}


def cascade_once(args, torch, Q, W, prec, seed_offset=0, timed=True):
    """One cascade run on a 2D Yee grid (2048 x 512 cells, 40 per wavelength, fp32 fields of
    a linearly polarised a0 = 300 pulse filled at t = 0): 1e6 electrons at gamma 4000 emit
    photons (NCS + Stokes), photons rotate their Stokes basis, evolve by vacuum
    birefringence and create pairs (NBW); electrons, positrons and photons all stepped in
    the order of the Spin-QED chain (qed_step), the leptons' current deposited and the field
    advanced by the Yee solver (open x boundaries) every step (the PIC loop; --no-deposit:
    vacuum solver, --static-grid: the snapshot at t = 0).  A warm-up builds the photon
    population, then the timed steps."""
    cfg = W.c3()
    grid, pulse = cfg["grid"], dict(cfg["pulse"])
    pulse["phi_start"] = -pulse["ncycles"] * math.pi          # pulse centre at x = 0 for t = 0
    comps = [torch.as_tensor(c).cuda() for c in W.grid_fill(grid, pulse, 0.0)]
    spec = dict(kind=Q.FIELD_GRID2D, grid=comps, **grid)
    n = len(cfg["leptons"]["x"])
    st = dict(cfg["leptons"])
    st["x"] = st["x"] - st["x"].mean()                          # bunch at the pulse centre
    precision = Q.QED_MIXED if prec == "mixed" else Q.QED_FP64
    ctx = Q.Context(dt=cfg["dt"], procs=cfg["procs"], seed=cfg["seed"] + seed_offset, id_start=cfg["next_id"],
                    precision=precision)
    cap_g, cap_l = 20_000_000, 4_000_000
    lists = {"em": Q.Leptons.from_state(st, capacity=cap_l, charge=-1, precision=precision),
             "ep": Q.Leptons(cap_l, 1, precision=precision), "G": Q.Photons(cap_g, precision=precision)}
    sort_every = args.sort_every
    # the lepton lists are short beside the photons' and feed the deposition, whose
    # 256-particle blocks want compact boxes: they may be sorted more often
    sort_lep = args.sort_leptons_every
    spare = ({"em": Q.Leptons(cap_l, -1, precision=precision), "ep": Q.Leptons(cap_l, 1, precision=precision),
              "G": Q.Photons(cap_g, precision=precision)} if (sort_every > 0 or sort_lep > 0) else None)
    segs = Q.whole(spec)
    warm, steps = args.cascade_warmup, args.cascade_steps
    solver = not args.static_grid
    deposit = solver and not args.no_deposit
    # the lists are kept in cell order by the periodic sort: the local deposition path
    dep_path = "local" if (sort_lep > 0 and args.deposit_path == "local") else "binned"
    ctx.set_deposit_path(Q.DEPOSIT_LOCAL if dep_path == "local" else Q.DEPOSIT_BINNED)
    # Jx, Jy, Jz: views of one array, cleared by one fill per step
    J_all = torch.zeros((3, grid["ny"], grid["nx"]), dtype=torch.float32, device="cuda")
    J = [J_all[0], J_all[1], J_all[2]]
    start = {"em": ctx.save_start(lists["em"]), "ep": ctx.save_start(lists["ep"])}

    def pic_step(s, ev=None):
        """every sort_every steps the photons, every sort_lep steps the leptons, reordered by
        grid bin (4 x 4 cells; dead photons dropped); save the lepton positions; the QED step in the order of the Spin-QED chain
        (pairs born this step are pushed and deposited from the next step on); current; field"""
        if ev: ev[0].record()
        if sort_every > 0 and s % sort_every == 0:
            ctx.sort_photons(lists["G"], spare["G"], spec, 4)
            lists["G"], spare["G"] = spare["G"], lists["G"]
        if sort_lep > 0 and s % sort_lep == 0:
            for k in ("em", "ep"):
                ctx.sort_leptons(lists[k], spare[k], spec, 4)
                lists[k], spare[k] = spare[k], lists[k]
        if ev: ev[1].record()
        em, ep, G = lists["em"], lists["ep"], lists["G"]
        if deposit:
            ctx.save_start(em, start["em"])
            ctx.save_start(ep, start["ep"])
        ctx.step(segs, em, ep, G, s)
        if ev: ev[2].record()
        if deposit:
            J_all.zero_()
            ctx.deposit_current([(em, start["em"]), (ep, start["ep"])], grid, J, CASCADE_QSCALE)
        if ev: ev[3].record()
        if solver:
            ctx.field_advance(spec, cfg["dt"], 1, current=J if deposit else None,
                              bc={"open_x": 1, "incoming": None, "gx0": grid["gx0"], "gy0": grid["gy0"],
                                  "t0": s * cfg["dt"]})
        if ev: ev[4].record()

    for s in range(warm):
        pic_step(s)
    torch.cuda.synchronize()
    # launch shape of the lepton step for these lists (far below their capacity)
    tuning = ctx.autotune(segs, lists["em"], warm, reps=2)
    counts0 = tuple(lists[k].count for k in ("em", "ep", "G"))
    # HIP events of every timed step (five around the step's parts, two around the photon
    # stage inside qed_step), read once after the loop: no synchronisation between steps,
    # so the host queues ahead of the device as in a production loop and no stage waits
    # for the host's launch of its first kernel
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(steps)]
    ph_ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(steps)]
    for e in [x for row in ev + ph_ev for x in row]:
        e.record()                 # creates the HIP event before the timed loop
    torch.cuda.synchronize()
    # what one timing marker itself adds to an interval: back-to-back records behind a busy
    # kernel (each interval between two events holds one such marker's own time)
    busy = torch.empty(1 << 26, dtype=torch.float32, device="cuda")
    busy.fill_(1.0)
    mk = [torch.cuda.Event(enable_timing=True) for _ in range(11)]
    for e in mk:
        e.record()
    torch.cuda.synchronize()
    marker_ms = sum(mk[i].elapsed_time(mk[i + 1]) for i in range(10)) / 10
    del busy
    t_ph = t_all = t_f = t_d = t_sort = 0.0
    t0 = time.perf_counter()
    for k, s in enumerate(range(warm, warm + steps)):
        if timed:
            ctx.set_photon_events(ph_ev[k])
        pic_step(s, ev[k] if timed else None)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.set_photon_events(None)
    if timed:
        for e, p in zip(ev, ph_ev):
            t_ph += p[0].elapsed_time(p[1])
            t_sort += e[0].elapsed_time(e[1])
            t_all += e[0].elapsed_time(e[4])
            t_d += e[2].elapsed_time(e[3])
            t_f += e[3].elapsed_time(e[4])
    em, ep, G = lists["em"], lists["ep"], lists["G"]
    counts1 = (em.count, ep.count, G.count)
    summary = cascade_summary(em, ep, G, 4000.0, torch)
    res = {"summary": summary, "counts0": counts0, "counts1": counts1, "status_bits": ctx.read_status(),
           "t_ph": t_ph, "t_all": t_all, "t_d": t_d, "t_f": t_f, "t_sort": t_sort, "sort_every": sort_every, "sort_lep": sort_lep,
           "wall": wall, "n": n, "warm": warm, "marker_ms": marker_ms,
           "steps": steps, "solver": solver, "deposit": deposit, "grid": grid, "tuning": tuning,
           "deposit_path": dep_path}
    ctx.close()
    del em, ep, G, J, J_all, comps, lists, spare
    torch.cuda.empty_cache()
    return res


def cascade_rates(r, prec):
    steps, counts0, counts1 = r["steps"], r["counts0"], r["counts1"]
    lep_steps = sum((counts0[k] + counts1[k]) / 2 * steps for k in (0, 1))
    pho_steps = (counts0[2] + counts1[2]) / 2 * steps
    ph_ms = r["t_ph"] / steps
    ph_bytes = (counts0[2] + counts1[2]) / 2 * BYTES_PHOTON_STEP[prec]
    gbs = ph_bytes / (ph_ms * 1e-3) / 1e9
    gbs_net = ph_bytes / ((ph_ms - r["marker_ms"]) * 1e-3) / 1e9
    return {"particle_steps_per_s": (lep_steps + pho_steps) / (r["t_all"] * 1e-3),
            "photon_steps_per_s": pho_steps / (r["t_ph"] * 1e-3),
            "ms_per_step": r["t_all"] / steps, "photon_step_ms": ph_ms, "wall_ms_per_step": 1e3 * r["wall"] / steps,
            "sort": {"every_steps": r["sort_every"], "leptons_every_steps": r["sort_lep"],
                     "ms_per_step": r["t_sort"] / steps,
                     "what": "photons (every_steps) and electrons, positrons (leptons_every_steps) reordered "
                             "by 4 x 4-cell grid bin (stable; dead photons dropped)"}
            if (r["sort_every"] or r["sort_lep"]) else None,
            "photon_step_roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                     "frac": gbs / HBM_PEAK_GBS, "bytes_per_photon_step": BYTES_PHOTON_STEP[prec],
                                     "frac_net_of_marker": gbs_net / HBM_PEAK_GBS},
            "timing_marker_ms": r["marker_ms"],
            "counts_start": {"electrons": counts0[0], "positrons": counts0[1], "photons": counts0[2]},
            "counts_end": {"electrons": counts1[0], "positrons": counts1[1], "photons": counts1[2],
                           "photons_alive": r["summary"]["photons_alive"]},
            "status_bits": r["status_bits"], "lepton_tuning": r["tuning"]}


def run_cascade(args, torch, Q, W):
    """The cascade in mixed precision (the timed result), the same run in FP64 (same draws)
    and FP64 with other draws: the mixed result stated at its error against FP64, each metric
    against max(4 x its difference between the two FP64 runs, 1e-3)."""
    mixed = cascade_once(args, torch, Q, W, "mixed")
    r = mixed
    if not args.cascade_mixed_only:
        fp64 = cascade_once(args, torch, Q, W, "fp64")
        fp64_b = cascade_once(args, torch, Q, W, "fp64", seed_offset=1, timed=False)
    steps, grid = r["steps"], r["grid"]
    nodes = grid["nx"] * grid["ny"]
    t_f, t_d = r["t_f"], r["t_d"]
    lep_mean = sum((r["counts0"][k] + r["counts1"][k]) / 2 for k in (0, 1))
    fgbs = nodes * BYTES_YEE_NODE / (t_f / steps * 1e-3) / 1e9 if r["solver"] and t_f > 0 else None
    dgbs = lep_mean * BYTES_DEPOSIT / (t_d / steps * 1e-3) / 1e9 if r["deposit"] and t_d > 0 else None
    field = ({"solver": ("2D Yee, open x (Mur) / periodic y, with the current the leptons deposit each step "
                         f"(charge-conserving, qscale {CASCADE_QSCALE})" if r["deposit"] else
                         "2D vacuum Yee, open x (Mur) / periodic y (the pulse filled at t = 0 and propagated)"),
              "ms_per_step": t_f / steps,
              "deposit": ({"ms_per_step": t_d / steps, "leptons": lep_mean,
                           "leptons_per_s": lep_mean / (t_d / steps * 1e-3),
                           "roofline": {"bound": "hbm", "achieved": dgbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                        "frac": dgbs / HBM_PEAK_GBS, "bytes_per_lepton": BYTES_DEPOSIT},
                           "path": r["deposit_path"],
                           "note": "includes zeroing J (the start positions are saved inside the QED step's interval)"}
                          if r["deposit"] else None),
              "roofline": {"bound": "hbm", "achieved": fgbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": fgbs / HBM_PEAK_GBS, "bytes_per_node_step": BYTES_YEE_NODE}}
             if r["solver"] else {"solver": "none (static snapshot of the pulse)"})
    out = {"workload": f"{r['n']} electrons gamma 4000 in an LP a0 = 300 pulse on a 2048 x 512 grid; "
                       f"NCS + Stokes + NBW + VB; steps {r['warm']}..{r['warm'] + steps - 1}",
           "field": field}
    out.update(cascade_rates(mixed, "mixed"))
    if args.cascade_mixed_only:
        return out
    err = cascade_metrics(fp64["summary"], mixed["summary"])
    stat = cascade_metrics(fp64["summary"], fp64_b["summary"])
    tol = {k: max(4.0 * stat[k], 1e-3) for k in CASCADE_DIFF}
    out["fp64"] = cascade_rates(fp64, "fp64")
    out["speedup_mixed_over_fp64"] = out["particle_steps_per_s"] / out["fp64"]["particle_steps_per_s"]
    out["error_vs_fp64"] = err
    out["error_statistical_fp64_seeds"] = stat
    out["tolerance_check"] = {"tolerance": tol, "within": {k: err[k] <= tol[k] for k in CASCADE_DIFF},
                              "all_within": all(err[k] <= tol[k] for k in CASCADE_DIFF)}
    return out


BYTES_HIST_PHOTON = {"mixed": 24 + 12 + 12 + 8 + 1, "fp64": 24 + 24 + 24 + 8 + 1}   # read k, xi, e1, w, alive


def run_detector(torch, Q, run, reps=5):
    """Detector histogram (qed_hist_photons) over the photon list the mixed headline run
    produced: angular map (p_y/p_x, p_z/p_x in +-10 mrad, 200 x 200) of counts, energy and
    the Stokes vector in the (y, z) detector basis; best of `reps` launches."""
    ctx, G = run["ctx"], run["G"]
    n = G.count
    h = Q.hist_spec((Q.AX_SLOPE_Y, Q.AX_SLOPE_Z), (200, 200), (-0.01, -0.01), (0.01, 0.01), (0, 1, 0))
    out = torch.zeros((200, 200, 5), dtype=torch.float64, device="cuda")
    best = float("inf")
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        out.zero_()
        a.record()
        ctx.hist_photons(G, 0, h, out=out)
        b.record()
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b))
    binned = float(out[..., 0].sum())
    gbs = n * BYTES_HIST_PHOTON["mixed"] / (best * 1e-3) / 1e9
    xi3 = float(out[..., 4].sum()) / max(binned, 1.0)
    return {"photons": n, "binned": binned, "ms": best, "photons_per_s": n / (best * 1e-3),
            "mean_xi3_detector": xi3,
            "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": gbs / HBM_PEAK_GBS, "bytes_per_photon": BYTES_HIST_PHOTON["mixed"]},
            "bins": "200 x 200 in p_y/p_x, p_z/p_x over +-10 mrad"}


BYTES_RADIATIVE = {"mixed": 48 + 12 + 48 + 12, "fp64": 48 + 24 + 48 + 24}   # read x, p, S; write x, p, S


def run_radiative(args, torch, Q, cfg):
    """Radiative push (MLL force + radiative T-BMT, qed_push_radiative) on the focused-pulse
    workload's 1e7 electrons at the peak field, mixed and FP64: throughput against the HBM
    roofline of its 120 / 144 algorithmic bytes per lepton-step, and the mean energy the
    radiation reaction removed."""
    out = {}
    mode = Q.RR_MLL | Q.RR_RBMT
    segs = Q.whole(cfg["field"])
    s0 = cfg["start_step"]
    for prec, name in ((Q.QED_MIXED, "mixed"), (Q.QED_FP64, "fp64")):
        ctx = Q.Context(dt=cfg["dt"], procs=cfg["procs"], seed=cfg["seed"], id_start=0, precision=prec)
        L = Q.Leptons.from_state(cfg["leptons"], precision=prec)
        n = L.count
        e0 = float(torch.sqrt(1 + L.px[:n] ** 2 + L.py[:n] ** 2 + L.pz[:n] ** 2).mean())
        for s in range(s0, s0 + 3):
            ctx.push_radiative(segs, L, mode, s)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * args.radiative_steps)]
        for k in range(args.radiative_steps):
            ev[2 * k].record()
            ctx.push_radiative(segs, L, mode, s0 + 3 + k)
            ev[2 * k + 1].record()
        torch.cuda.synchronize()
        ms = sum(ev[2 * k].elapsed_time(ev[2 * k + 1]) for k in range(args.radiative_steps)) / args.radiative_steps
        e1 = float(torch.sqrt(1 + L.px[:n] ** 2 + L.py[:n] ** 2 + L.pz[:n] ** 2).mean())
        gbs = n * BYTES_RADIATIVE[name] / (ms * 1e-3) / 1e9
        out[name] = {"lepton_steps_per_s": n / (ms * 1e-3), "ms_per_step": ms,
                     "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                  "frac": gbs / HBM_PEAK_GBS, "bytes_per_lepton_step": BYTES_RADIATIVE[name]},
                     "mean_gamma_change_rel": e1 / e0 - 1, "status_bits": ctx.read_status()}
    out["mode"] = "MLL force + radiative T-BMT"
    out["workload"] = "1e7 electrons, focused CP pulse a0 = 100, gamma0 = 2000, steps from 2400"
    return out


# bremsstrahlung decide kernel per electron-step in the target: read x, p (32 B) and the id
# (8 B) for the draws; an emitting electron is re-read and written by the event kernel
BYTES_BREMS = 8 + 24 + 8


def run_brems(args, torch, Q):
    """Bremsstrahlung in a target (Sec. III.E): the paper's check configuration, 1e5
    electrons of 1 GeV normally incident on 5 mm of gold and of aluminium (field-free push +
    bremsstrahlung step until every electron has left the slab, photons above 1 MeV), with
    the mean energy left against the radiation-length estimate exp(-L / X0); and the step's
    throughput on 1e7 electrons inside gold (mixed and FP64) against the HBM roofline of its
    decide kernel."""
    import numpy as np
    out = {}
    um = 1e-6 / (2 * math.pi)                       # length unit c / omega_L at 1 um, metres
    mev = 1.0 / 0.51099895
    thick = 5e-3 / um
    targets = {"Au": (79, 5.90e28, 0.3344), "Al": (13, 6.026e28, 8.897)}   # Z, atoms / m^3, X0 (cm)
    dt = 20.0
    n = 100_000
    E0 = 1000.0 * mev
    for name, (Z, dens, x0_cm) in targets.items():
        ctx = Q.Context(dt=dt, procs=0, seed=5, id_start=0, precision=Q.QED_FP64, p_max=1.0)
        ctx.brems_init(Z, dens * um ** 3, 0.0, thick, 1.0 * mev)
        pz = math.sqrt(E0 * E0 - 1.0)
        st = {"x": np.zeros(n), "y": np.zeros(n), "z": np.zeros(n), "px": np.full(n, pz), "py": np.zeros(n),
              "pz": np.zeros(n), "w": np.ones(n), "sx": np.zeros(n), "sy": np.zeros(n), "sz": np.zeros(n),
              "id": np.arange(n, dtype=np.uint64)}
        L = Q.Leptons.from_state(st)
        G = Q.Photons(40 * n)
        segs = Q.whole({"kind": Q.FIELD_NONE})
        steps = int(thick / dt) + 2
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(steps):
            ctx.push_spin(segs, L, s)
            ctx.step_brems(L, G, s)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        e = torch.sqrt(1 + L.px[:n] ** 2 + L.py[:n] ** 2 + L.pz[:n] ** 2)
        k = torch.sqrt(G.kx[:G.count] ** 2 + G.ky[:G.count] ** 2 + G.kz[:G.count] ** 2)
        out[name] = {"photons_per_electron": G.count / n, "mean_energy_left": float(e.mean()) / E0,
                     "radiation_length_estimate": math.exp(-0.5 / x0_cm),
                     "photon_energy_fraction": float(k.sum()) / (n * E0),
                     "photons_above_100MeV_per_electron": float((k > 100 * mev).sum()) / n,
                     "steps": steps, "wall_s": wall, "status_bits": ctx.read_status()}
    # throughput: 1e7 electrons of 100 MeV..10 GeV inside gold, the step alone
    nt = 10_000_000
    g = np.random.default_rng(11)
    Ee = np.exp(g.uniform(math.log(100 * mev), math.log(1e4 * mev), nt))
    st = {"x": g.uniform(0.0, thick, nt), "y": np.zeros(nt), "z": np.zeros(nt), "px": np.sqrt(Ee * Ee - 1.0),
          "py": np.zeros(nt), "pz": np.zeros(nt), "w": np.ones(nt), "sx": np.zeros(nt), "sy": np.zeros(nt),
          "sz": np.zeros(nt), "id": np.arange(nt, dtype=np.uint64)}
    for prec, pname in ((Q.QED_MIXED, "mixed"), (Q.QED_FP64, "fp64")):
        ctx = Q.Context(dt=dt, procs=0, seed=6, id_start=0, precision=prec, p_max=1.0)
        ctx.brems_init(79, 5.90e28 * um ** 3, 0.0, thick, 1.0 * mev)
        L = Q.Leptons.from_state(st, precision=prec)
        G = Q.Photons(nt // 2, precision=prec)
        ctx.step_brems(L, G, 0)
        torch.cuda.synchronize()
        c0 = G.count
        K = args.brems_steps
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * K)]
        for j in range(K):
            ev[2 * j].record()
            ctx.step_brems(L, G, 1 + j)
            ev[2 * j + 1].record()
        torch.cuda.synchronize()
        ms = sum(ev[2 * j].elapsed_time(ev[2 * j + 1]) for j in range(K)) / K
        gbs = nt * BYTES_BREMS / (ms * 1e-3) / 1e9
        out["throughput_" + pname] = {
            "electron_steps_per_s": nt / (ms * 1e-3), "ms_per_step": ms, "photons_per_step": (G.count - c0) / K,
            "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": gbs / HBM_PEAK_GBS, "bytes_per_electron_step": BYTES_BREMS,
                         "note": "whole step (decide + scan + events) against the decide kernel's bytes"},
            "status_bits": ctx.read_status()}
        del L, G
    out["workload"] = ("1e5 electrons of 1 GeV through 5 mm of Au and of Al (k > 1 MeV, dt = 20 c/omega_L); "
                       "1e7 electrons of 100 MeV..10 GeV inside Au for the throughput")
    return out


def _oracle_run(st, cfg, steps, budget_s=None):
    """The oracle as it stands (C, FP64 tables) on the electrons `st`: `steps` steps, or as
    many as `budget_s` seconds allow (at most `steps`).  Returns (particle-steps, seconds)."""
    import oracle
    n = len(st["x"])
    L = oracle.LeptonArrays.from_state(st)
    G = oracle.PhotonArrays.empty(int(0.03 * n * steps) + 1000)
    sim = oracle.Sim(dt=cfg["dt"], procs=cfg["procs"], seed=cfg["seed"], next_id=cfg["next_id"])
    f = oracle.make_field(cfg["field"])
    s0 = cfg["start_step"]
    done = 0
    t0 = time.perf_counter()
    while done < steps and (budget_s is None or time.perf_counter() - t0 < budget_s):
        sim.step(f, L, None, G, s0 + done)
        done += 1
    return n * done, time.perf_counter() - t0


_CPU_JOB = {}


def _cpu_worker(k):
    """One process of the all-core baseline: slice k of the sample, a fixed step count."""
    job = _CPU_JOB
    m = job["per"]
    st = {key: v[k * m:(k + 1) * m] for key, v in job["cfg"]["leptons"].items()}
    return _oracle_run(st, job["cfg"], job["steps"])


def cpu_baseline(W, start, n1=200_000, budget_s=15.0):
    """The oracle as it stands, timed on the host cores, before this process touches the
    GPU: (1) single-threaded on the first n1 electrons of the bunch, stepped until the budget
    is used; (2) one process per core of the machine's CPU share (at most 16), each stepping its
    own n1 electrons (disjoint slices of a larger bunch of the same recipe) for the same
    number of steps.  Particles are independent and the draws are keyed by particle id, so
    the processes need no communication; the rate is all particle-steps over the wall time
    of the slowest process."""
    import multiprocessing as mp
    import oracle
    oracle.build()
    oracle.tables()
    nproc = os.cpu_count() or 1
    try:
        share = len(os.sched_getaffinity(0))
    except AttributeError:
        share = nproc
    ncores = max(1, min(16, share))
    cfg = W.c2(n1 * ncores, start_step=start)
    st1 = {k: v[:n1] for k, v in cfg["leptons"].items()}
    ps, el = _oracle_run(st1, cfg, 400, budget_s)
    steps = max(1, ps // n1)
    single = {"value": ps / el, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
              "sample": f"{n1} electrons of the focused-pulse bunch x {steps} steps from step {start} "
                        f"(single-threaded C oracle, FP64 tables), {el:.1f} s"}
    _CPU_JOB.update(cfg=cfg, per=n1, steps=steps)
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(ncores) as pool:   # forked before any GPU use
        res = pool.map(_cpu_worker, range(ncores))
    wall = time.perf_counter() - t0
    _CPU_JOB.clear()
    total = sum(r[0] for r in res)
    return {"value": total / wall, "unit": "particle-steps/s", "cores": ncores, "kind": "oracle",
            "sample": f"{ncores} processes x {n1} electrons (disjoint slices of a {n1 * ncores}-electron bunch of "
                      f"the focused-pulse recipe) x {steps} steps from step {start}, {wall:.1f} s wall "
                      f"(slowest process {max(r[1] for r in res):.1f} s)",
            "host": {"nproc": nproc, "cpu_share": share, "processes": ncores},
            "single_core": single}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=10_000_000, help="electrons (default: the full workload)")
    ap.add_argument("--cpu-sample", type=int, default=200_000)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--batch-steps", type=int, default=50,
                    help="steps of the many-collision batching comparison (0: skip it)")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-sampler measurements")
    ap.add_argument("--cascade-steps", type=int, default=40, help="timed steps of the cascade (0: skip it)")
    ap.add_argument("--cascade-warmup", type=int, default=150)
    ap.add_argument("--sort-every", type=int, default=20,
                    help="cascade: reorder the particle lists by grid bin every N steps (0: never)")
    ap.add_argument("--sort-leptons-every", type=int, default=10,
                    help="cascade: reorder the lepton lists by grid bin every N steps (0: never)")
    ap.add_argument("--cascade-mixed-only", action="store_true",
                    help="cascade: only the timed mixed-precision run (no FP64 runs, no error metrics)")
    ap.add_argument("--full-steps", type=int, default=6000,
                    help="steps of the whole-interaction accuracy leg (0: skip it)")
    ap.add_argument("--full-n", type=int, default=1_000_000, help="electrons of the whole-interaction leg")
    ap.add_argument("--deposit-path", choices=("local", "binned"), default="local",
                    help="cascade: deposition path for the cell-ordered lists (binned: any order)")
    ap.add_argument("--no-deposit", action="store_true",
                    help="cascade: vacuum field solver, no current deposition")
    ap.add_argument("--static-grid", action="store_true",
                    help="cascade on a static snapshot of the pulse instead of the Yee-propagated field")
    ap.add_argument("--radiative-steps", type=int, default=20,
                    help="timed steps of the radiative push (MLL + radiative T-BMT; 0: skip it)")
    ap.add_argument("--train-samples", type=int, default=10_000_000)
    ap.add_argument("--brems-steps", type=int, default=20,
                    help="timed bremsstrahlung steps on 1e7 electrons (0: skip the bremsstrahlung leg)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device to device three times (a plain copy kernel of known size, "
                         "the reference for the HBM byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark measures one GPU; the particle step shards by index "
                                   "range with no per-step communication, and no multi-GPU run is part of it",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    cpu = None
    if not args.no_cpu_baseline and not args.copy_probe:
        import workloads as W
        print("[bench] CPU baseline (oracle), single core and all cores, before the GPU is used",
              file=sys.stderr, flush=True)
        cpu = cpu_baseline(W, 2400 + args.warmup, args.cpu_sample, args.cpu_budget)
        print(f"[bench] CPU baseline: {cpu['value']:.3e} particle-steps/s on {cpu['cores']} cores, "
              f"{cpu['single_core']['value']:.3e} on one", file=sys.stderr, flush=True)

    import torch

    if args.copy_probe:
        nbytes = args.copy_probe << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):   # an elementwise kernel (x * 1): reads and writes nbytes each
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": nbytes, "copy_probe_bytes_written": nbytes,
                          "kernel": "torch elementwise x * 1.0 in float64 (MulFunctor), 3 dispatches"}))
        return

    import paper_2306_11288_amd as Q
    import workloads as W

    torch.cuda.set_device(0)
    start = 2400
    cfg = W.c2(args.n, start_step=start)
    print(f"[bench] workload {cfg['name']} n={args.n} steps={args.steps} warmup={args.warmup}", file=sys.stderr,
          flush=True)
    mixed = run_gpu("mixed", cfg, args.steps, args.warmup, torch, Q)
    print(f"[bench] mixed done: {args.steps * args.n / mixed['wall']:.3e} particle-steps/s", file=sys.stderr,
          flush=True)
    fp64 = fp64_b = None
    if not args.no_fp64:
        fp64 = run_gpu("fp64", cfg, args.steps, args.warmup, torch, Q)
        print(f"[bench] fp64 done: {args.steps * args.n / fp64['wall']:.3e} particle-steps/s", file=sys.stderr,
              flush=True)
        # the same run with other random draws: the statistical spread of the error metrics
        fp64_b = run_gpu("fp64", dict(cfg, seed=cfg["seed"] + 1), args.steps, args.warmup, torch, Q,
                         per_launch_events=False)

    ms_per_step = 1e3 * mixed["wall"] / args.steps
    value = args.n * args.steps / mixed["wall"]
    km = {k: sum(v) / len(v) for k, v in mixed["kern_ms"].items()}
    ph_per_launch = mixed["photons_timed"] / args.steps
    # the dominant kernel is the decide kernel: every lepton, 128 algorithmic bytes each
    alg_bytes = args.n * BYTES_LEPTON["mixed"]
    achieved = alg_bytes / (km["decide"] * 1e-3) / 1e9
    step_bytes = alg_bytes + ph_per_launch * BYTES_PHOTON["mixed"]
    tr = measured_traffic("mixed")
    copy_gbs = copy_bandwidth(torch)
    result = {
        "metric": "particle-steps/s (push+spin+QED) mixed vs FP64 GPU at stated spectrum error",
        "value": value, "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64 (x, p, event probability, field phase f64; fields, rates, sampling, spin, Stokes f32)",
        "data": "synthetic (seeded numpy Philox bunch; analytic focused pulse)",
        "config": {"workload": "c2_focused_cp_pulse_a0_100_1e7_electrons_gamma2000", "electrons": args.n,
                   "gamma0": 2000, "a0": 100, "w0_um": 3.0, "ncycles": 10, "dt": "T0/500",
                   "start_step": start, "processes": "NCS + spin flip + photon Stokes"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": tr,
                     "kernel": "k_leptons_decide<float, push, gauss>", "tuning": mixed["tuning"],
                     "avg_launch_ms": km["decide"], "algorithmic_bytes_per_launch": alg_bytes,
                     "copy_probe_GBs": copy_gbs, "frac_of_copy_probe": achieved / copy_gbs,
                     "step_ms": {"decide": km["decide"], "scan": km["scan"], "events": km["events"],
                                 "step": km["step"]},
                     "step_algorithmic_GBs": step_bytes / (km["step"] * 1e-3) / 1e9,
                     "photons_per_launch": ph_per_launch,
                     "events": f"HIP events around the launches of every {EV_EVERY}th timed step "
                               f"({len(mixed['kern_ms']['decide'])} steps); each interval includes one "
                               "event record's own device time (a few microseconds)"},
        "status_bits": mixed["status"],
    }
    if fp64 is not None:
        fk = {k: sum(v) / len(v) for k, v in fp64["kern_ms"].items()}
        result["fp64"] = {"value": args.n * args.steps / fp64["wall"], "ms_per_step": 1e3 * fp64["wall"] / args.steps,
                          "decide_ms": fk["decide"], "step_ms": fk["step"],
                          "decide_achieved_GBs": args.n * BYTES_LEPTON["fp64"] / (fk["decide"] * 1e-3) / 1e9,
                          "status_bits": fp64["status"]}
        result["speedup_mixed_over_fp64"] = result["value"] / result["fp64"]["value"]
        result["error_vs_fp64"] = error_metrics(fp64, mixed, 2000.0, torch)
        stat = error_metrics(fp64, fp64_b, 2000.0, torch)
        result["error_statistical_fp64_seeds"] = stat
        result["error_tolerance"] = tolerance_check(result["error_vs_fp64"], stat)
    print("[bench] detector histogram", file=sys.stderr, flush=True)
    result["detector"] = run_detector(torch, Q, mixed)
    if args.radiative_steps > 0:
        print("[bench] radiative push", file=sys.stderr, flush=True)
        result["radiative"] = run_radiative(args, torch, Q, cfg)
    if args.brems_steps > 0:
        print("[bench] bremsstrahlung", file=sys.stderr, flush=True)
        result["brems"] = run_brems(args, torch, Q)
    if args.cascade_steps > 0:
        print("[bench] cascade on the grid", file=sys.stderr, flush=True)
        result["cascade"] = run_cascade(args, torch, Q, W)
    if not args.no_learned:
        print("[bench] learned sampler", file=sys.stderr, flush=True)
        result["learned"] = run_learned(args, torch, Q, W, cfg, fp64, fp64_b)
    if args.batch_steps > 0:
        print("[bench] batching: many collisions, graph-replayed, vs one at a time in FP64", file=sys.stderr, flush=True)
        result["batched"] = run_batched(args, torch, Q, W)
    if args.full_steps > 0:
        print("[bench] the whole interaction, mixed vs FP64", file=sys.stderr, flush=True)
        result["full_interaction"] = run_full_interaction(args, torch, Q, W)
    if cpu is not None:
        result["cpu_baseline"] = cpu
    print(json.dumps(result))


if __name__ == "__main__":
    main()
