#!/usr/bin/env python3
"""Throughput of the WENO-IS finite-volume RK3 stage on one MI355X.

Workload: the 2D shock-bubble problem at 1024 x 512 cells (air cylinder in
water hit by a 1 GPa water shock; workloads.shock_bubble_2d), MOOD on,
CFL 0.5 time step recomputed on the device every step.  A step is one full
RK3 step: the time-step reduction plus three stages, each stage a complete
evaluation of the hot path (primitive recovery, characteristic projection,
WENO-IS, MOOD cascade, HLLC, flux difference, Runge-Kutta update) over the
whole grid.

Metric: cell-updates per second per RK stage = cells * 3 * steps / time,
inputs resident in HBM before the timed region.  `value` is the plain FP64
path; the FP32 reconstruction/flux form is timed the same way and reported
with its L1 difference from the FP64 path after the same steps.

Printed: ONE JSON line (rank 0).  --gpus > 1 is refused: the path runs on
a single GPU (how it would shard is described with the design).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

# Algorithmic operations of the method per unit (add, multiply, divide,
# square root and comparison each one), as the oracle's operation counter
# counts them on the oracle's own evaluation (structural zeros and ones of
# the face matrices free, a repeated operation counted once, a discarded
# value not counted; the test suite checks these figures against it):
#   face (smooth, subsonic, no fallback): averaged state 8, face matrices
#   10, projection of six cells 36, (10 + nt) WENO-IS values of 101 less 25
#   shared between the two sides, back-projection 16, positivity 6, HLLC
#   99 + 8 nt (nt = ndim - 1 transverse velocities);
#   cell: primitive recovery, per axis the flux difference and sources
#   (2 nc + 7, plus nc to add the earlier axes' terms), Runge-Kutta update.
FACE_OPS = {1: 1160, 2: 1269, 3: 1378}
# A reconstruction that takes its shortcut (FP64: tau5 of eq. (25) exactly
# zero, so the weights are exactly d_k: candidates 16, tau5 15, combination
# 7, the test 1 = 39 of the 101 operations; FP32 form: a flat stencil, its
# spread 8 operations) saves the difference.
SHORTCUT_SAVING_F64 = 101 - 39
SHORTCUT_SAVING_F32 = 101 - 8
PRIM_OPS = {1: 7, 2: 10, 3: 13}
UPDATE_OPS_PER_STEP = {1: 58, 2: 70, 3: 82}   # three stages per cell


def axis_ops(nd, d):
    nc = 4 + nd
    return 2 * nc + 7 + (nc if d > 0 else 0)


# Algorithmic HBM bytes per cell and stage: read U_s and write U_{s+1}
# (8 bytes x nc each), plus U^n in stages 2 and 3 (2/3 on average).
def BYTES_PER_CELL_STAGE(nd):
    nc = 4 + nd
    return 8 * nc * (2 + 2 / 3)


# Published MI355X peaks: vector FP64 78.6 and FP32 157.3 TFLOP/s (an FMA
# counted as two operations, FP32 also as packed pairs), HBM3E 8 TB/s.
# `roofline.frac` is taken against these.
PEAK = {"f64_valu_tflops": 78.6, "f32_valu_tflops": 157.3, "hbm_gbs": 8000.0}
# The same vector units without fused multiply-add or packed math:
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3e12 operations per second,
# FP64 and FP32 alike.  The stage kernels are built without contraction or
# packed FP32 (the FP64 path reproduces the oracle's rounding), so every
# algorithmic add, multiply, divide or square root costs at least one
# instruction and 39.3e12 op/s is the ceiling they can reach; reported next
# to the published figure as `frac_no_fma`.
VALU_OPS_PEAK_T = 256 * 4 * 16 * 2.4e9 / 1e12

HERE = os.path.dirname(os.path.abspath(__file__))
STAGE_SOURCES = ("face.hpp", "sweep.hpp", "sweep_kernels.hpp", "kernels.hip", "sweep_f32.hip",
                 "stage2d_kernel.hpp", "stage2d.hip", "stage2d_f32.hip")
COUNTERS_FILE = os.path.join(HERE, "profiles", "stage_2d_shock_bubble_1024x512_counters.md")
COUNTERS_3D = os.path.join(HERE, "profiles", "sweep_3d_shock_droplet_256_counters.md")


def measured_traffic(kernel, counters_file=None):
    """HBM bytes per launch of `kernel` from a committed counter summary
    (default: the 2D benchmark's), or None when the stage-kernel sources
    have changed since it was taken."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in STAGE_SOURCES:
        with open(os.path.join(HERE, "paper_1707_00592_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    try:
        text = open(counters_file or COUNTERS_FILE).read()
    except OSError:
        return None
    m = re.search(r"stage-kernel sources: ([0-9a-f]{16})", text)
    t = re.search(r"traffic %s bytes_per_launch: (\d+)" % kernel, text)
    if not m or not t or m.group(1) != h.hexdigest()[:16]:
        return None
    return int(t.group(1))


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--nx", type=int, default=1024)
    ap.add_argument("--ny", type=int, default=512)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--forms", default="fp64,fp32,cutoff",
                    help="forms of the main workload: fp64 (the headline), fp32, cutoff")
    ap.add_argument("--full-steps", type=int, default=1000,
                    help="steps of the full-run report (the workload as configured); 0 skips it")
    ap.add_argument("--skip", type=int, default=0,
                    help="advance the initial state by this many untimed FP64 steps first "
                         "(for profiling developed states; 0 for the benchmark)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a 512 MiB device copy (reference for HBM counters)")
    ap.add_argument("--extras", default="config1,mlp,accuracy,study,mood,paper2d,3d,batch",
                    help="other workloads to report: config1 (the 200-cell gas-liquid shock "
                         "tube), mlp (learned weights, trained here), "
                         "accuracy (every form against a 2x finer FP64 run), study (basic, "
                         "modified and cut-off weights, 1D convergence), mood (cost of the "
                         "MOOD cascade where fallbacks are common), paper2d (the paper's 2D "
                         "cylinder, droplet and bubble cases at full size), 3d (256^3 "
                         "shock-droplet), batch (4096 uneven tubes); empty for none")
    ap.add_argument("--steps-3d", type=int, default=200,
                    help="steps of the 3D shock-droplet workload (its configuration: 200)")
    ap.add_argument("--t-end-steps", type=int, default=1000,
                    help="the learned-weights workload runs to the time the 1024x512 FP64 run "
                         "reaches in this many steps (its configuration: 1000)")
    return ap.parse_args()


def l1_rel(a, b):
    return float((a - b).abs().sum() / b.abs().sum())


def run_steps(isweno, ctx, p, U0, opts, steps, warmup, torch):
    """Untimed warmup, then `steps` RK3 steps; returns (U, seconds, stats)."""
    grid = isweno.make_grid(p.n, p.dx, p.bc_lo, p.bc_hi)
    U = U0.clone()
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    st = isweno.new_stats()
    for _ in range(warmup):
        ctx.rk3_step(U, grid, opts, dt, st)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.rk3_step(U, grid, opts, dt, st)
    torch.cuda.synchronize()
    return U, time.perf_counter() - t0, isweno.read_stats(st)


def extra_3d(isweno, workloads, ctx, torch, steps=200):
    """3D shock-droplet 256^3, FP32 reconstruction with FP64 recovery, next
    to the FP64 path on the same steps: throughput, per-kernel times over
    every step (a second, directly launched pass), the HBM roofline from
    algorithmic bytes and, while the stage sources match the committed
    counter summary, the measured HBM bytes of each sweep."""
    p = workloads.shock_droplet_3d(256)
    U0 = torch.from_numpy(p.U).to("cuda")
    del p.U
    out = {"workload": "3D shock-droplet 256^3, MOOD on, CFL 0.5", "steps": steps}
    res = {}
    for name, prec in (("fp32", isweno.FP32), ("fp64", isweno.FP64)):
        U, el, kern, st, _ = run_form(isweno, ctx, p, U0, isweno.make_opts(precision=prec),
                                      steps, 2, torch)
        v = p.ncells * 3 * steps / el
        bw = v * BYTES_PER_CELL_STAGE(3) / 1e9
        res[name] = U
        for k, rec in kern.items():
            t = measured_traffic(f"{name} {k}", COUNTERS_3D)
            if t is not None:
                rec["traffic_bytes_per_launch"] = t
                rec["hbm_at_traffic_gbs"] = round(t / (rec["avg_ms"] * 1e-3) / 1e9, 1)
        out[name] = {"value": v, "unit": "cell-updates/s per RK stage", "status": st.status,
                     "kernels": kern,
                     "hbm_roofline": {"bound": "hbm", "achieved": round(bw, 1),
                                      "peak": PEAK["hbm_gbs"], "unit": "GB/s",
                                      "frac": round(bw / PEAK["hbm_gbs"], 4),
                                      "bytes_per_cell_stage": round(BYTES_PER_CELL_STAGE(3), 1)}}
        traffic = [r.get("traffic_bytes_per_launch") for k, r in kern.items()
                   if k.startswith("sweep")]
        if traffic and all(t is not None for t in traffic):
            # measured bytes of a stage (x, y and z sweeps) against the
            # algorithmic bytes of a stage
            per_stage = sum(traffic)
            out[name]["hbm_roofline"]["traffic"] = per_stage
            out[name]["hbm_roofline"]["traffic_over_algorithmic"] = round(
                per_stage / (p.ncells * BYTES_PER_CELL_STAGE(3)), 3)
        else:
            out[name]["hbm_roofline"]["traffic"] = None
    out["fp32"]["speedup_vs_fp64"] = out["fp32"]["value"] / out["fp64"]["value"]
    out["fp32"]["l1_rel_rho_vs_fp64"] = l1_rel(res["fp32"][0], res["fp64"][0])
    del res, U0
    torch.cuda.empty_cache()
    return out


def extra_paper2d(isweno, workloads, ctx, torch, steps=300):
    """The paper's 2D workloads at the paper's finest grids: the air-R22 and
    air-He cylinders at 3000 x 1000 between walls (MOOD off), the air-water
    droplet at 800 x 800 (MOOD off) and the water-air bubble at 1600 x 1600
    (MOOD on); FP64 and FP32, `steps` CFL steps each from the start."""
    cases = [("air_R22_3000x1000", lambda: workloads.shock_gas_cylinder_2d("R22"), False),
             ("air_He_3000x1000", lambda: workloads.shock_gas_cylinder_2d("He"), False),
             ("air_water_droplet_800x800", lambda: workloads.air_water_2d("droplet", 800), False),
             ("water_air_bubble_1600x1600", lambda: workloads.air_water_2d("bubble", 1600), True)]
    out = {"steps": steps}
    for name, make, mood in cases:
        p = make()
        U0 = torch.from_numpy(p.U).to("cuda")
        r = {"cells": p.ncells, "mood": mood}
        res = {}
        for form, prec in (("fp64", isweno.FP64), ("fp32", isweno.FP32)):
            U, el, st = run_steps(isweno, ctx, p, U0,
                                  isweno.make_opts(precision=prec, mood=mood), steps, 2, torch)
            res[form] = U
            r[form] = {"value": p.ncells * 3 * steps / el, "status": st.status,
                       "mood_o3": list(st.o3[:2]), "mood_o1": list(st.o1[:2])}
        r["fp32"]["speedup_vs_fp64"] = r["fp32"]["value"] / r["fp64"]["value"]
        r["fp32"]["l1_rel_rho_vs_fp64"] = l1_rel(res["fp32"][0], res["fp64"][0])
        if p.bc_lo[1] == 2:
            # symmetric about the channel axis: v odd, the rest even
            nx, ny = p.n
            u = res["fp64"].view(6, ny, nx)
            m = u.flip(1).clone()
            m[2] = -m[2]
            scale = u.abs().amax(dim=(1, 2))
            diff = (u - m).abs().amax(dim=(1, 2))
            keep = scale > 0
            r["fp64"]["mirror_asymmetry"] = float((diff[keep] / scale[keep]).max())
        out[name] = r
        del res, U0
        torch.cuda.empty_cache()
    return out


def extra_batch(isweno, workloads, ctx, torch, steps=100):
    """4096 uneven two-phase shock tubes, one HIP graph per RK3 step,
    autotuned tiles; FP64 and FP32."""
    b = workloads.batch_riemann(4096, seed=1707)
    total = int(b["offsets"][-1])
    U0 = torch.from_numpy(b["U"]).to("cuda")
    plan = ctx.batch_plan(b["offsets"], b["dx"])
    out = {"workload": f"4096 uneven 1D two-phase shock tubes ({total} cells)", "steps": steps}
    res = {}
    for name, prec in (("fp64", isweno.FP64), ("fp32", isweno.FP32)):
        opts = isweno.make_opts(precision=prec)
        tile = plan.autotune(U0, opts)
        U = U0.clone()
        dt = torch.zeros(4096, dtype=torch.float64, device="cuda")
        st = isweno.new_stats()
        plan.reset_status()
        plan.step(U, opts, dt, 2, st)            # capture the graph, warm up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.step(U, opts, dt, steps, st)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        res[name] = U
        frozen = (plan.status != 0).nonzero().flatten().cpu().tolist()
        out[name] = {"value": total * 3 * steps / el, "unit": "cell-updates/s per RK stage",
                     "tile": tile, "frozen_problems": frozen,
                     "note": "value counts every cell; frozen problems (non-physical, "
                             "stopped individually) are listed"}
    out["fp32"]["speedup_vs_fp64"] = out["fp32"]["value"] / out["fp64"]["value"]
    ok = torch.ones(total, dtype=torch.bool, device="cuda")
    for k in set(out["fp64"]["frozen_problems"]) | set(out["fp32"]["frozen_problems"]):
        ok[int(b["offsets"][k]):int(b["offsets"][k + 1])] = False
    out["fp32"]["l1_rel_rho_vs_fp64"] = l1_rel(res["fp32"][0][ok], res["fp64"][0][ok])
    plan.close()
    return out


def config2_t_end(isweno, workloads, ctx, torch, nsteps=1000):
    """The time the 1024 x 512 shock-bubble (FP64, CFL 0.5) reaches in its
    configured 1000 steps: the final time of the workload at every
    resolution and form."""
    p = workloads.shock_bubble_2d(1024, 512)
    g = isweno.make_grid(p.n, p.dx, p.bc_lo, p.bc_hi)
    U = torch.from_numpy(p.U).to("cuda")
    _, t_end, _ = isweno.Solver(g, isweno.make_opts(), ctx).run(U, nsteps=nsteps, t_end=1.0)
    return t_end


def extra_mlp(isweno, workloads, ctx, torch, t_end):
    """Learned weights: trained on the GPU on faces of plain runs of the
    gas-liquid shock tube and the 3D shock-droplet (at 96^3), then run on
    the 2D shock-bubble at 2048 x 1024 to the final time of the 1000-step
    1024 x 512 workload (t_end), next to the FP64 and FP32 forms.  Each form
    runs twice from the initial state: once to t_end exactly (the last step
    clipped; the state compared), once timed over the same number of steps
    as HIP-graph replays.  Returns (report, packed network)."""
    from paper_1707_00592_amd import learned
    t0 = time.perf_counter()
    opts64 = isweno.make_opts()
    X, Y = learned.collect(ctx, [workloads.sod_gas_liquid(200)], opts64, steps=250, every=10,
                           stride=1, max_rows=20000)
    X3, Y3 = learned.collect(ctx, [workloads.shock_droplet_3d(96, radius_cells=12.0)], opts64,
                             steps=100, every=20, stride=29, max_rows=1_000_000)
    X = torch.cat([X, X3]); Y = torch.cat([Y, Y3])
    Xs, Ys = learned.stratify(X, Y, limit=4_000_000)
    P, hist = learned.train(ctx, Xs, Ys, steps=3000, batch=65536, lr=3e-3, log_every=500)
    ev = learned.evaluate(ctx, P, Xs, Ys)
    train_s = time.perf_counter() - t0
    packed = torch.zeros(isweno.MLP_NPARAM, dtype=torch.int16, device="cuda")
    ctx.mlp_pack(P, packed)
    p2 = workloads.shock_bubble_2d(2048, 1024)
    g2 = isweno.make_grid(p2.n, p2.dx, p2.bc_lo, p2.bc_hi)
    U2 = torch.from_numpy(p2.U).to("cuda")
    forms = {"fp64": isweno.make_opts(),
             "fp32": isweno.make_opts(precision=isweno.FP32),
             "mlp": learned_opts(isweno, packed)}
    out = {"workload": "2D shock-bubble 2048x1024, MOOD on, CFL 0.5", "t_end": t_end}
    res = {}
    for name, o in forms.items():
        U = U2.clone()
        st = isweno.new_stats()
        _, t, k = isweno.Solver(g2, o, ctx).run(U, t_end=t_end, stats=st)
        st = isweno.read_stats(st)
        res[name] = U
        # learned face-fields (the four non-material fields) of those k steps
        faces = sum(p2.ncells // p2.n[d] * (p2.n[d] + 1) for d in range(2)) * 4 * 3 * k
        _, el, kern, _, _ = run_form(isweno, ctx, p2, U2, o, k, 0, torch, 20)
        out[name] = {"value": p2.ncells * 3 * k / el, "unit": "cell-updates/s per RK stage",
                     "steps": k, "status": st.status, "kernels": kern,
                     "mood": {"o3": list(st.o3[:2]), "o1": list(st.o1[:2])}}
        if name == "mlp":
            out[name]["fallback_rate"] = float(sum(st.mlp_fallback[:2])) / faces
    pref = pressure(res["fp64"])
    for name in ("fp32", "mlp"):
        out[name]["speedup_vs_fp64"] = out[name]["value"] / out["fp64"]["value"]
        out[name]["l1_rel_rho_vs_fp64"] = l1_rel(res[name][0], res["fp64"][0])
        out[name]["l1_rel_p_vs_fp64"] = l1_rel(pressure(res[name]), pref)
    out["mlp"]["speedup_vs_fp32"] = out["mlp"]["value"] / out["fp32"]["value"]
    out["note"] = ("the FP64 path equals the oracle bit for bit (parity tests), so its state is "
                   "the FP64 reference of the L1 figures")
    out["training"] = {"samples": int(Xs.shape[0]), "adam_steps": 3000,
                       "seconds": round(train_s, 1), "loss": hist, **ev}
    del res, U2
    torch.cuda.empty_cache()
    return out, packed


def extra_config1(isweno, workloads, ctx, torch):
    """The 200-cell gas-liquid shock tube (MOOD off, as in Sec. 5) to
    t = 2.4e-4 s: launch-bound at this size; timed as graph replays of the
    step count the run to t_end takes."""
    p = workloads.sod_gas_liquid(200)
    g = isweno.make_grid(p.n, p.dx, p.bc_lo, p.bc_hi)
    out = {"workload": "1D gas-liquid shock tube, 200 cells, t_end 2.4e-4 s"}
    for name, prec in (("fp64", isweno.FP64), ("fp32", isweno.FP32)):
        o = isweno.make_opts(precision=prec, mood=False)
        U = torch.from_numpy(p.U).to("cuda")
        _, t, k = isweno.Solver(g, o, ctx).run(U, t_end=p.t_end)
        U0 = torch.from_numpy(p.U).to("cuda")
        _, el, _, st, _ = run_form(isweno, ctx, p, U0, o, k, 5, torch, 5)
        out[name] = {"steps": k, "value": p.ncells * 3 * k / el,
                     "unit": "cell-updates/s per RK stage", "ms_per_step": el / k * 1e3,
                     "status": st.status}
    return out


def learned_opts(isweno, packed):
    return isweno.make_opts(precision=isweno.FP32, weights=isweno.W_MLP, mlp_params=packed,
                            mlp_conf_threshold=0.5)


def pressure(U):
    """p = (E - rho |u|^2 / 2 - Pi) / Gamma of a 2D state [6][N]."""
    rho = U[0]
    ke = 0.5 * (U[1] * U[1] + U[2] * U[2]) / rho
    return (U[3] - ke - U[5]) / U[4]


def equal_l1(isweno, workloads, ctx, torch, forms, values, nsteps=1000):
    """Each form on the 1024x512 shock-bubble to the time the FP64 path
    reaches in `nsteps` steps, against the FP64 path at 2048x1024 averaged
    over 2x2 blocks: L1 of rho and p per form, and whether it lies within 5%
    of the FP64 form's L1 (the condition under which the speed-ups are
    quoted at equal error)."""
    p = workloads.shock_bubble_2d(1024, 512)
    g = isweno.make_grid(p.n, p.dx, p.bc_lo, p.bc_hi)
    U = torch.from_numpy(p.U).to("cuda")
    _, t_end, _ = isweno.Solver(g, forms["fp64"], ctx).run(U.clone(), nsteps=nsteps, t_end=1.0)
    pr = workloads.shock_bubble_2d(2048, 1024)
    gr = isweno.make_grid(pr.n, pr.dx, pr.bc_lo, pr.bc_hi)
    Ur = torch.from_numpy(pr.U).to("cuda")
    isweno.Solver(gr, forms["fp64"], ctx).run(Ur, t_end=t_end)
    ref = Ur.view(6, 512, 2, 1024, 2).mean(dim=(2, 4)).reshape(6, -1)
    del Ur
    pref = pressure(ref)
    out = {"t_end": t_end, "reference": "FP64 path at 2048x1024, 2x2 block averages"}
    for name, o in forms.items():
        Uf = U.clone()
        isweno.Solver(g, o, ctx).run(Uf, t_end=t_end)
        out[name] = {"l1_rho": float((Uf[0] - ref[0]).abs().mean() / ref[0].abs().mean()),
                     "l1_p": float((pressure(Uf) - pref).abs().mean() / pref.abs().mean())}
        if name in values:
            out[name]["value"] = values[name]
    base = out["fp64"]
    for name in forms:
        f = out[name]
        f["equal_l1"] = bool(abs(f["l1_rho"] - base["l1_rho"]) <= 0.05 * base["l1_rho"] and
                             abs(f["l1_p"] - base["l1_p"]) <= 0.05 * base["l1_p"])
        if "value" in f and "value" in base:
            f["speedup_vs_fp64"] = f["value"] / base["value"]
    return out


def run_form(isweno, ctx, p, U0, opts, steps, warmup, torch, kernel_steps=None):
    """Warmup, then `steps` timed RK3 steps (each a replay of the step's
    HIP graph); then, from the same start and after the same warmup, the
    first `kernel_steps` (default: all) of those steps again, launched
    directly with every kernel bracketed by HIP events on its stream
    (per-kernel durations on the states the timed steps saw)."""
    grid = isweno.make_grid(p.n, p.dx, p.bc_lo, p.bc_hi)
    U = U0.clone()
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    st = isweno.new_stats()
    for _ in range(warmup):
        ctx.rk3_step(U, grid, opts, dt, st)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.rk3_step(U, grid, opts, dt, st)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    stats = isweno.read_stats(st)
    Uk = U0.clone()
    ks = steps if kernel_steps is None else kernel_steps
    dk = torch.zeros(1, dtype=torch.float64, device="cuda")
    sk = isweno.new_stats()
    for _ in range(warmup):
        ctx.rk3_step(Uk, grid, opts, dk, sk)
    ctx.timing_enable(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(ks):
        ctx.rk3_step(Uk, grid, opts, dk, sk)
    torch.cuda.synchronize()
    el_direct = time.perf_counter() - t1
    kern = {}
    shortcuts = ctx.shortcut_read()
    for k, name in isweno.K_NAMES.items():
        ms, n = ctx.timing_read(k)
        if n:
            kern[name] = {"total_ms": ms, "launches": n, "avg_ms": ms / n}
            if k < 3:
                kern[name]["shortcuts_per_launch"] = shortcuts[k] / n
            elif k == isweno.K_STAGE2D:
                # the fused 2D stage counts its x and y field-sides per axis
                kern[name]["shortcuts_per_launch"] = (shortcuts[0] + shortcuts[1]) / n
    ctx.timing_enable(False)
    del Uk
    return U, el, kern, stats, {"steps": ks, "ms_per_step": el_direct / ks * 1e3}


def kernel_work(name, p):
    """(axes, faces, cells, algorithmic operations, algorithmic HBM bytes) of
    one launch of stage kernel `name` on problem p, before shortcuts.  A
    launch of "stage_2d" is a whole 2D stage (x and y faces, the cell
    updates); a sweep launch is one axis (the last axis also does the
    Runge-Kutta update).  Bytes: the state read and the stage written, plus
    U^n in stages 2 and 3 (two thirds on average); a sweep that is not the
    last reads or writes the partial sum instead, which the method does not
    need, so only the fused stage's bytes are algorithmic per launch."""
    nd = p.ndim
    cells = p.ncells
    nc = 4 + nd
    if name == "stage_2d":
        axes = [0, 1]
    else:
        axes = [{"sweep_x": 0, "sweep_y": 1, "sweep_z": 2}[name]]
    faces = sum(cells // p.n[D] * (p.n[D] + 1) for D in axes)
    ops = faces * FACE_OPS[nd] + cells * sum(axis_ops(nd, D) for D in axes)
    ops += cells * PRIM_OPS[nd] * len(axes)
    if axes[-1] == nd - 1:
        ops += cells * UPDATE_OPS_PER_STEP[nd] / 3
    hbm = cells * BYTES_PER_CELL_STAGE(nd) if len(axes) == nd else None
    return axes, faces, cells, ops, hbm, nc


def full_run(isweno, ctx, p, U0, opts, steps, torch):
    """The workload as configured: `steps` RK3 steps from the initial state
    (graph replays, one untimed step first to capture the graph, then the
    state reset in place), then the same steps again with every kernel
    timed, so that per-kernel figures cover the whole run rather than its
    quiescent start."""
    grid = isweno.make_grid(p.n, p.dx, p.bc_lo, p.bc_hi)
    U = U0.clone()
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    st = isweno.new_stats()
    ctx.rk3_step(U, grid, opts, dt, st)
    U.copy_(U0)
    dt.zero_()
    st.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.rk3_step(U, grid, opts, dt, st)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    stats = isweno.read_stats(st)
    Uk = U0.clone()
    dk = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.timing_enable(True)
    for _ in range(steps):
        ctx.rk3_step(Uk, grid, opts, dk)
    torch.cuda.synchronize()
    kern = {}
    shortcuts = ctx.shortcut_read()
    for k, name in isweno.K_NAMES.items():
        ms, n = ctx.timing_read(k)
        if n:
            kern[name] = {"total_ms": ms, "launches": n, "avg_ms": ms / n}
            if k < 3:
                kern[name]["shortcuts_per_launch"] = shortcuts[k] / n
            elif k == isweno.K_STAGE2D:
                kern[name]["shortcuts_per_launch"] = (shortcuts[0] + shortcuts[1]) / n
    ctx.timing_enable(False)
    same = bool(torch.equal(U, Uk))
    del Uk
    return U, el, kern, stats, same


def roofline(kern, p, precision, with_traffic=False):
    """Dominant kernel's achieved rate of algorithmic operations against the
    published vector peak of its precision (frac), next to the no-FMA
    ceiling (frac_no_fma, see VALU_OPS_PEAK_T) and to HBM (hbm_frac, the
    algorithmic bytes of a whole stage over the launch time)."""
    name, k = max(((n, v) for n, v in kern.items() if n.startswith(("sweep", "stage"))),
                  key=lambda kv: kv[1]["total_ms"])
    axes, faces, cells, flops, hbm, nc = kernel_work(name, p)
    # reconstructions that took their shortcut did less work
    sc = k.get("shortcuts_per_launch", 0.0)
    saving = SHORTCUT_SAVING_F64 if precision == "f64" else SHORTCUT_SAVING_F32
    flops -= sc * saving
    sec = k["avg_ms"] * 1e-3
    achieved = flops / sec / 1e12
    peak = PEAK["f64_valu_tflops"] if precision == "f64" else PEAK["f32_valu_tflops"]
    # the committed counters cover the timed window from the initial state
    traffic = None
    if with_traffic:
        traffic = measured_traffic(name if precision == "f64" else "fp32 " + name)
    out = {"bound": "alu", "kernel": name, "achieved": round(achieved, 3), "peak": peak,
           "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": traffic,
           "peak_no_fma": round(VALU_OPS_PEAK_T, 1),
           "frac_no_fma": round(achieved / VALU_OPS_PEAK_T, 4),
           "flops_per_launch": int(flops), "avg_launch_ms": round(k["avg_ms"], 4),
           "launches": k["launches"],
           "shortcut_fraction": round(sc / (faces * 2 * nc), 4),
           "flops_per_launch_without_shortcuts": int(flops + sc * saving),
           "hbm_at_traffic_gbs": None if traffic is None else round(traffic / sec / 1e9, 1)}
    if hbm is not None:
        out["hbm_algorithmic_gbs"] = round(hbm / sec / 1e9, 1)
        out["hbm_frac"] = round(hbm / sec / 1e9 / PEAK["hbm_gbs"], 4)
        out["hbm_bytes_per_launch"] = int(hbm)
    return out


def cpu_baseline(p, seconds):
    """The oracle (plain FP64 C, OpenMP) on the same workload: the first RK3
    steps until about `seconds` of CPU work on every host thread, then about
    a quarter of that on one thread for a per-core figure."""
    import oracle

    def sample(budget, max_steps):
        g = oracle.make_grid(p.n, p.dx, p.bc_lo, p.bc_hi)
        o = oracle.make_opts(mood=True, cfl=0.5)
        U = p.U.copy()
        steps = 0
        t0 = time.perf_counter()
        while True:
            h = oracle.cfl_dt(U, g, o)
            U, s = oracle.rk3_step(U, g, h, o)
            steps += 1
            el = time.perf_counter() - t0
            if el >= budget or steps >= max_steps:
                return steps, el

    all_threads = oracle.threads()
    steps, el = sample(seconds, 200)
    oracle.threads(1)
    steps1, el1 = sample(seconds / 4, 200)
    oracle.threads(all_threads)
    return {"value": p.ncells * 3 * steps / el, "unit": "cell-updates/s per RK stage",
            "cores": all_threads, "kind": "oracle",
            "sample": f"first {steps} RK3 steps of the {p.n[0]}x{p.n[1]} shock-bubble "
                      f"({steps * 3 * p.ncells} cell-stages, {el:.1f} s)",
            "per_core_value": p.ncells * 3 * steps1 / el1,
            "per_core_sample": f"first {steps1} RK3 steps on one thread ({el1:.1f} s)"}


def form_opts(isweno, f):
    """Options of a named form of the main workload: fp64 (the method), fp32
    (float reconstruction and flux), cutoff (FP64 with the targeted-ENO
    cut-off weights)."""
    prec = isweno.FP32 if f == "fp32" else isweno.FP64
    w = isweno.W_CUTOFF if f == "cutoff" else isweno.W_MODIFIED
    return isweno.make_opts(precision=prec, weights=w, mood=True, cfl=0.5)


def progress(msg, t0=None):
    """One line on stderr as each part of the run ends (the JSON line is
    the only output on stdout)."""
    tail = "" if t0 is None else f" ({time.perf_counter() - t0:.1f} s)"
    print(f"bench.py: {msg}{tail}", file=sys.stderr, flush=True)


def rel_l1(a, b):
    return float((a - b).abs().sum() / b.abs().sum())


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: runs on one GPU only; --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(3)
    from paper_1707_00592_amd import isweno, workloads
    isweno.load()
    p = workloads.shock_bubble_2d(args.nx, args.ny)
    U0 = torch.from_numpy(p.U).to("cuda")
    ctx = isweno.Context(0)
    if args.skip > 0:
        g0 = isweno.make_grid(p.n, p.dx, p.bc_lo, p.bc_hi)
        d0 = torch.zeros(1, dtype=torch.float64, device="cuda")
        for _ in range(args.skip):
            ctx.rk3_step(U0, g0, isweno.make_opts(), d0)
        torch.cuda.synchronize()
    forms = [f.strip() for f in args.forms.split(",") if f.strip()]
    results = {}
    for f in forms:
        t0 = time.perf_counter()
        opts = form_opts(isweno, f)
        U, el, kern, st, direct = run_form(isweno, ctx, p, U0, opts, args.steps, args.warmup,
                                           torch)
        results[f] = {"U": U, "elapsed": el, "kern": kern, "stats": st, "direct": direct}
        progress(f"timed steps, {f}", t0)
    base = results["fp64"]
    cells_stages = p.ncells * 3 * args.steps
    value = cells_stages / base["elapsed"]
    out = {
        "metric": "cell-updates/s per RK stage",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": base["elapsed"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"2D shock-bubble {p.n[0]}x{p.n[1]}, FP64, MOOD on, CFL 0.5",
                   "cells": p.ncells, "rk_stages_per_step": 3, "parallelism": "single GPU"},
        "roofline": roofline(base["kern"], p, "f64", with_traffic=True),
        "kernels": base["kern"],
        "kernel_timing_pass": dict(base["direct"], note="kernel durations come from a second "
                                   "pass over the same steps from the same start, launched "
                                   "directly (no graph) with HIP events around every kernel"),
        "mood": {"o3": list(base["stats"].o3[:2]), "o1": list(base["stats"].o1[:2]),
                 "status": base["stats"].status},
    }
    out["roofline"]["hbm_frac_of_value"] = round(
        value * BYTES_PER_CELL_STAGE(p.ndim) / 1e9 / PEAK["hbm_gbs"], 4)
    # The timed window above is the start of the run (quiescent water ahead
    # of the shock, most reconstructions on the linear-weight shortcut);
    # the workload as configured is 1000 steps, which the shock needs to
    # cross the bubble.  Report it too, per form.
    nfull = args.full_steps
    full = {"steps": nfull, "note": f"{nfull} RK3 steps from the initial state (graph "
            "replays), per-kernel figures from a second, directly launched pass over the same "
            "steps"}
    full_U = {}
    for f in (forms if nfull > 0 else []):
        o = form_opts(isweno, f)
        t0 = time.perf_counter()
        Uf, el, kern, st, same = full_run(isweno, ctx, p, U0, o, nfull, torch)
        progress(f"full run, {f}", t0)
        full_U[f] = Uf
        full[f] = {"value": p.ncells * 3 * nfull / el,
                   "kernels": kern,
                   "roofline": (roofline(kern, p, "f32" if f == "fp32" else "f64")
                                if f != "cutoff" else None),
                   "mood": {"o3": list(st.o3[:2]), "o1": list(st.o1[:2]), "status": st.status},
                   "timing_pass_bitwise_equal": same}
        full[f]["ms_per_step"] = el / nfull * 1e3
        full[f]["hbm_frac_of_value"] = round(
            full[f]["value"] * BYTES_PER_CELL_STAGE(p.ndim) / 1e9 / PEAK["hbm_gbs"], 4)
    for f in full_U:
        if f == "fp64" or "fp64" not in full_U:
            continue
        full[f]["speedup_vs_fp64"] = full[f]["value"] / full["fp64"]["value"]
        full[f]["l1_rel_rho_vs_fp64"] = rel_l1(full_U[f][0], full_U["fp64"][0])
        full[f]["l1_rel_p_vs_fp64"] = rel_l1(pressure(full_U[f]), pressure(full_U["fp64"]))
    if nfull > 0:
        out["config_full_run"] = full
    del full_U
    rho64 = base["U"][0]
    forms_out = {}
    for f, r in results.items():
        if f == "fp64":
            continue
        v = cells_stages / r["elapsed"]
        forms_out[f] = {"value": v, "speedup_vs_fp64": v / value,
                        "l1_rel_rho_vs_fp64": rel_l1(r["U"][0], rho64),
                        "l1_rel_E_vs_fp64": rel_l1(r["U"][3], base["U"][3]),
                        "status": r["stats"].status,
                        "kernels": r["kern"]}
        if f == "fp32":
            # (the operation counts are those of the eq. (28) weights: no
            # roofline line for the cut-off form)
            forms_out[f]["roofline"] = roofline(r["kern"], p, "f32", with_traffic=True)
    extras = [e.strip() for e in args.extras.split(",") if e.strip()]
    out["forms"] = forms_out
    other = {}
    packed = None
    if "config1" in extras:
        t0 = time.perf_counter()
        try:
            other["gas_liquid_tube_200"] = extra_config1(isweno, workloads, ctx, torch)
        except Exception as e:  # report, keep the contract line
            other["gas_liquid_tube_200"] = {"error": repr(e)}
        progress("config1", t0)
    if "mlp" in extras:
        t0 = time.perf_counter()
        try:
            t_end = config2_t_end(isweno, workloads, ctx, torch, args.t_end_steps)
            other["learned_weights"], packed = extra_mlp(isweno, workloads, ctx, torch, t_end)
            o = learned_opts(isweno, packed)
            nfull = max(args.full_steps, 1)
            Uf, el, kern, st, _ = full_run(isweno, ctx, p, U0, o, nfull, torch)
            faces = sum(p.ncells // p.n[d] * (p.n[d] + 1) for d in range(2)) * 4 * 3 * nfull
            forms_out["mlp"] = {"value": p.ncells * 3 * nfull / el, "steps": nfull,
                                "note": f"{nfull} steps from the initial state (the configured "
                                        "run), as config_full_run",
                                "status": st.status, "kernels": kern,
                                "fallback_rate": float(sum(st.mlp_fallback[:2])) / faces}
            forms_out["mlp"]["speedup_vs_fp64"] = forms_out["mlp"]["value"] / (
                out["config_full_run"]["fp64"]["value"] if "config_full_run" in out else value)
            del Uf
        except Exception as e:  # report, keep the contract line
            other["learned_weights"] = {"error": repr(e)}
        progress("mlp", t0)
    if "accuracy" in extras:
        t0 = time.perf_counter()
        try:
            fo = {"fp64": isweno.make_opts(), "fp32": isweno.make_opts(precision=isweno.FP32)}
            vals = {"fp64": value}
            if "fp32" in forms_out:
                vals["fp32"] = forms_out["fp32"]["value"]
            if packed is not None:
                fo["mlp"] = learned_opts(isweno, packed)
                vals["mlp"] = forms_out["mlp"]["value"]
            other["equal_l1_1024x512"] = equal_l1(isweno, workloads, ctx, torch, fo, vals)
        except Exception as e:
            other["equal_l1_1024x512"] = {"error": repr(e)}
        progress("accuracy", t0)
    if "study" in extras:
        t0 = time.perf_counter()
        try:
            from paper_1707_00592_amd import studies
            other["weights_study_1d"] = studies.weights_study(ctx)
        except Exception as e:
            other["weights_study_1d"] = {"error": repr(e)}
        progress("study", t0)
    if "mood" in extras:
        t0 = time.perf_counter()
        try:
            from paper_1707_00592_amd import studies
            other["mood_cost"] = studies.mood_cost_study(ctx)
        except Exception as e:
            other["mood_cost"] = {"error": repr(e)}
        progress("mood", t0)
    if "paper2d" in extras:
        t0 = time.perf_counter()
        try:
            other["paper_2d"] = extra_paper2d(isweno, workloads, ctx, torch)
        except Exception as e:
            other["paper_2d"] = {"error": repr(e)}
        progress("paper2d", t0)
    if "3d" in extras:
        t0 = time.perf_counter()
        try:
            other["shock_droplet_3d"] = extra_3d(isweno, workloads, ctx, torch, args.steps_3d)
        except Exception as e:
            other["shock_droplet_3d"] = {"error": repr(e)}
        progress("3d", t0)
    if "batch" in extras:
        t0 = time.perf_counter()
        try:
            other["batch_riemann"] = extra_batch(isweno, workloads, ctx, torch)
        except Exception as e:
            other["batch_riemann"] = {"error": repr(e)}
        progress("batch", t0)
    if other:
        out["other_workloads"] = other
    if not args.no_cpu:
        t0 = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(p, args.cpu_seconds)
        progress("cpu baseline", t0)
    if args.copy_probe:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE per
        # dispatch scale the counters of the stage kernels to bytes
        a = torch.empty(64 << 20, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = {"read": a.numel() * 8, "write": b.numel() * 8}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
