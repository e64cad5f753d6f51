"""Training driver of the learned nonlinear weights (not in the paper).

Data: face samples that the method itself generates.  Plain WENO-IS runs of
given problems are snapshotted and isweno_mlp_samples turns every face and
characteristic field into 8 network inputs plus the eq. (28) weights of both
sides (the targets).  Samples whose candidate values (eq. (20), on the
normalised stencil) spread by more than 0.05 of the stencil's range on a
side, where the weights decide the result, are kept whole; the rest, where
any convex weights give nearly the same value, is thinned so that the former
make up a stated share.

Loss: the error of the value the predicted weights reconstruct against the
value of the target weights (both on the same candidates), plus a
confidence head trained to say whether that error is below 0.005 of the
stencil's range; in the solver, faces below the confidence threshold use the
eq. (28) weights.

Training: full-precision float32 master parameters, bf16 matrix-core
forward and backward (isweno_mlp_loss_grad), Adam (isweno_mlp_adam), all in
the library; this module only selects data and loops.
"""
from __future__ import annotations

import math

import numpy as np

from . import isweno

def init_params(seed: int = 1707) -> np.ndarray:
    """He-uniform weights, zero biases; the confidence bias starts at +2."""
    rs = np.random.default_rng(seed)
    P = np.zeros(isweno.MLP_NPARAM, dtype=np.float32)
    o = 0
    for fan_out, fan_in in ((32, 8), (32, 32), (9, 32)):
        lim = math.sqrt(6.0 / fan_in)
        P[o:o + fan_out * fan_in] = rs.uniform(-lim, lim, fan_out * fan_in)
        o += fan_out * fan_in + fan_out
    P[-1] = 2.0
    return P


def collect(ctx: isweno.Context, problems, opts: isweno.Opts, steps: int, every: int,
            stride: int, max_rows: int):
    """Runs each workload.Problem with the plain path for `steps` RK3 steps
    and samples its faces every `every` steps.  Returns (X, Y) cuda tensors."""
    import torch
    Xs, Ys = [], []
    for p in problems:
        grid = isweno.make_grid(p.n, p.dx, p.bc_lo, p.bc_hi)
        U = torch.from_numpy(np.ascontiguousarray(p.U)).to("cuda")
        dt = torch.zeros(1, dtype=torch.float64, device="cuda")
        count = torch.zeros(1, dtype=torch.int64, device="cuda")
        for k in range(steps + 1):
            if k % every == 0:
                X = torch.empty((max_rows, 8), dtype=torch.float32, device="cuda")
                Y = torch.empty((max_rows, 8), dtype=torch.float32, device="cuda")
                ctx.mlp_samples(U, grid, opts, X, Y, max_rows, stride, count)
                m = int(count.item())
                Xs.append(X[:m]); Ys.append(Y[:m])
            if k < steps:
                ctx.rk3_step(U, grid, opts, dt)
    return torch.cat(Xs), torch.cat(Ys)


def candidates(X):
    """Candidates of eq. (20) of both sides on the normalised stencils
    X[:, 0..5]: returns (left [n,4], right [n,4])."""
    import torch

    def c4(a, b, c, d, e):
        return torch.stack([0.5 * c + 0.5 * d, -0.5 * b + 1.5 * c,
                            c / 3.0 + 5.0 * d / 6.0 - e / 6.0,
                            a / 3.0 - 7.0 * b / 6.0 + 11.0 * c / 6.0], dim=1)
    x = X
    return (c4(x[:, 0], x[:, 1], x[:, 2], x[:, 3], x[:, 4]),
            c4(x[:, 5], x[:, 4], x[:, 3], x[:, 2], x[:, 1]))


def stratify(X, Y, share_nontrivial: float = 0.3, seed: int = 1707, limit: int | None = None):
    """Keeps every sample whose candidates spread by more than 0.05 on a side
    and enough of the others that the former are `share_nontrivial` of the
    set (or all of them if there are too few of the others)."""
    import torch
    cl, cr = candidates(X)
    spread = torch.maximum(cl.amax(1) - cl.amin(1), cr.amax(1) - cr.amin(1))
    nontriv = spread > 0.05
    gen = torch.Generator(device="cpu").manual_seed(seed)
    idx_n = torch.nonzero(nontriv).flatten().cpu()
    idx_t = torch.nonzero(~nontriv).flatten().cpu()
    want_t = int(len(idx_n) * (1 - share_nontrivial) / share_nontrivial)
    if want_t < len(idx_t):
        idx_t = idx_t[torch.randperm(len(idx_t), generator=gen)[:want_t]]
    idx = torch.cat([idx_n, idx_t])
    idx = idx[torch.randperm(len(idx), generator=gen)]
    if limit is not None:
        idx = idx[:limit]
    idx = idx.to(X.device)
    return X[idx].contiguous(), Y[idx].contiguous()


def train(ctx: isweno.Context, X, Y, steps: int = 2000, batch: int = 65536, lr: float = 3e-3,
          seed: int = 1707, params=None, log_every: int = 0):
    """Adam on mini-batches (fixed order, seeded shuffle).  Returns
    (params float32 cuda tensor, list of (step, loss))."""
    import torch
    P = torch.from_numpy(init_params(seed) if params is None else np.asarray(params, np.float32))
    P = P.to("cuda").contiguous()
    g = torch.zeros_like(P); m = torch.zeros_like(P); v = torch.zeros_like(P)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    n = X.shape[0]
    gen = torch.Generator(device="cpu").manual_seed(seed)
    order = torch.randperm(n, generator=gen).to(X.device)
    hist = []
    pos = 0
    for k in range(1, steps + 1):
        if pos + batch > n:
            order = torch.randperm(n, generator=gen).to(X.device)
            pos = 0
        sel = order[pos:pos + batch]
        pos += batch
        xb = X[sel].contiguous(); yb = Y[sel].contiguous()
        ctx.mlp_loss_grad(P, xb, yb, None, loss, g)
        ctx.mlp_adam(P, g, m, v, k, lr)
        if log_every and (k % log_every == 0 or k == 1):
            hist.append((k, float(loss.item())))
    return P, hist


def evaluate(ctx: isweno.Context, P, X, Y, conf_threshold: float = 0.5):
    """Value error of the predicted weights on a set (units of the stencil's
    range): its mean, the share of samples within 0.005 on both sides, the
    share the confidence head accepts, and the share of accepted samples
    that are within 0.005 (precision of the confidence head)."""
    import torch
    out = torch.empty((X.shape[0], 9), dtype=torch.float32, device="cuda")
    ctx.mlp_forward(P, X, out)
    pl = torch.softmax(out[:, :4], dim=1); pr = torch.softmax(out[:, 4:8], dim=1)
    cl, cr = candidates(X)
    el = ((pl - Y[:, :4]) * cl).sum(1).abs()
    er = ((pr - Y[:, 4:]) * cr).sum(1).abs()
    err = torch.maximum(el, er)
    ok = err < 0.005
    conf = torch.sigmoid(out[:, 8]) >= conf_threshold
    acc = float((ok & conf).float().sum() / conf.float().sum().clamp(min=1.0))
    return {"mean_value_err": float(err.mean()), "frac_within_0.005": float(ok.float().mean()),
            "frac_confident": float(conf.float().mean()), "confident_precision": acc}
