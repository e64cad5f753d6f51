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
