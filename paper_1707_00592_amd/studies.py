"""Accuracy study of the nonlinear-weight forms on the GPU path.

The paper motivates its modified weights (eq. (28)) by the loss of accuracy
of the basic form (eq. (21)) at critical points of smooth data.  This runs
the smooth entropy wave (a sine, with extrema, and the Gauss pulse of eqs.
(33)-(34)) on the GPU with both forms, at dt = 0.5 dx^(5/3) as in Sec. 4,
and reports the L1 error of the density against the exact cell averages
and the observed orders.  The cut-off form (the targeted-ENO optimisation
the conclusions propose, Sec. 7) runs next to them, also over one full
period of the pulse, where the dissipation of smooth data adds up.
"""
from __future__ import annotations

import math

import numpy as np

from . import isweno, workloads


def entropy_errors(ctx: isweno.Context, ns, weights: int, pulse: bool, t_end: float = 0.1,
                   amp: float = 0.2, precision: int = isweno.FP64):
    """L1 and max errors of rho after t_end on the periodic unit interval."""
    import torch
    out = []
    for n in ns:
        p = workloads.entropy_wave(n, 1, amp=amp, pulse=pulse)
        g = isweno.make_grid(p.n, p.dx, p.bc_lo, p.bc_hi)
        dx = 1.0 / n
        steps = int(math.ceil(t_end / (0.5 * dx ** (5.0 / 3.0))))
        o = isweno.make_opts(precision=precision, weights=weights, mood=False, cfl=0.0)
        U = torch.from_numpy(np.ascontiguousarray(p.U)).to("cuda")
        dt = torch.full((1,), t_end / steps, dtype=torch.float64, device="cuda")
        for _ in range(steps):
            ctx.rk3_step(U, g, o, dt)
        exact = workloads.exact_entropy_average(p.n, t_end, amp, pulse)
        e = np.abs(U[0].cpu().numpy() - exact)
        out.append((float(e.mean()), float(e.max())))
    return out


FORMS = (("modified", isweno.W_MODIFIED), ("basic", isweno.W_BASIC),
         ("cutoff", isweno.W_CUTOFF))


def weights_study(ctx: isweno.Context):
    """The weight forms on the sine and the pulse (t = 0.1), and on the
    pulse carried once around the domain (t = 1, the smooth-region
    dissipation the cut-off form is for); errors and orders."""
    res = {}
    for name, pulse, ns, t_end in (("sine", False, [20, 40, 80, 160], 0.1),
                                   ("pulse", True, [50, 100, 200, 400], 0.1),
                                   ("pulse_period", True, [50, 100, 200], 1.0)):
        for form, w in FORMS:
            e = entropy_errors(ctx, ns, w, pulse, t_end=t_end)
            l1 = np.array([x[0] for x in e])
            res[f"{name}_{form}"] = {"n": ns, "t_end": t_end, "l1": l1.tolist(),
                                     "max": [x[1] for x in e],
                                     "orders": np.log2(l1[:-1] / l1[1:]).round(2).tolist()}
    return res


def mood_cost_study(ctx: isweno.Context, fracs=(0.0, 0.001, 0.01, 0.1, 1.0), reps: int = 20):
    """Cost of the MOOD cascade (Sec. 3.4) where its fallbacks are common.

    The 1024 x 512 shock-bubble start state with a fraction of its cells
    replaced by independent random two-phase states (water or air, |u|, |v|
    up to 2000 m/s, p from 1e4 to 3e9 Pa): one FP64 RHS (the fused 2D
    stage kernel) timed with the cascade on and off, with the fallback
    counts, and with the gathered cascade (mood = 2).  The redo of a failing
    face side is a divergent branch inside its wave, so its cost follows the
    waves that hold a failing side, not the failing sides themselves."""
    import torch
    base = workloads.shock_bubble_2d(1024, 512)
    g = isweno.make_grid(base.n, base.dx, base.bc_lo, base.bc_hi)
    sides = 2 * ((base.n[0] + 1) * base.n[1] + base.n[0] * (base.n[1] + 1))
    rs = np.random.default_rng(1707)
    out = {"workload": "2D shock-bubble 1024x512 start state, a fraction of the cells "
                       "replaced by random two-phase states; one FP64 RHS",
           "reps": reps, "rows": []}
    for f in fracs:
        U = base.U.copy()
        m = rs.random(base.ncells) < f
        k = int(m.sum())
        if k:
            rho = np.where(rs.random(k) < 0.5, 1000.0, 1.0) * rs.uniform(0.5, 2.0, k)
            water = rho > 100.0
            vel = [rs.uniform(-2000.0, 2000.0, k), rs.uniform(-2000.0, 2000.0, k)]
            p = 10.0 ** rs.uniform(4.0, 9.5, k)
            U[:, m] = workloads.prim_to_cons(rho, vel, p, np.where(water, 4.4, 1.4),
                                             np.where(water, 6e8, 0.0))
        Ud = torch.from_numpy(np.ascontiguousarray(U)).to("cuda")
        row = {"fraction": f, "cells": k}
        for mood in (isweno.MOOD_ON, isweno.MOOD_OFF, isweno.MOOD_GATHER):
            o = isweno.make_opts(mood=mood)
            ctx.rhs(Ud, g, o)                       # warm
            torch.cuda.synchronize()
            st = isweno.new_stats()
            ctx.timing_enable(True)
            for _ in range(reps):
                ctx.rhs(Ud, g, o, stats=st)
            torch.cuda.synchronize()
            ms, n = ctx.timing_read(isweno.K_STAGE2D)
            ctx.timing_enable(False)
            s = isweno.read_stats(st)
            key = {isweno.MOOD_ON: "mood_on", isweno.MOOD_OFF: "mood_off",
                   isweno.MOOD_GATHER: "mood_gathered"}[mood]
            row[key] = {"stage_us": 1e3 * ms / n}
            if mood == isweno.MOOD_ON:
                o3 = sum(s.o3[:2]) / reps
                o1 = sum(s.o1[:2]) / reps
                row[key].update({"order3_sides": o3, "order1_sides": o1,
                                 "fallback_fraction": (o3 + o1) / sides})
        row["cascade_cost_us"] = row["mood_on"]["stage_us"] - row["mood_off"]["stage_us"]
        row["gathered_cascade_cost_us"] = (row["mood_gathered"]["stage_us"]
                                           - row["mood_off"]["stage_us"])
        out["rows"].append(row)
        del Ud
    return out
