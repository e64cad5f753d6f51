"""Training driver of the learned nonlinear weights (not in the paper).

Data: face samples that the method itself generates.  Plain WENO-IS runs of
given problems are snapshotted and isweno_mlp_samples turns every face and
characteristic field into 8 network inputs plus the eq. (28) weights of both
sides (the targets).  Samples whose target weights leave the optimal weights
d_k (0.4, 0.2, 0.3, 0.1) by more than 0.05 on a side, where the nonlinear
weights act, are kept whole; the rest is thinned so that the former make up
a stated share.

Loss: the error of the value the predicted weights reconstruct against the
value of the target weights (both on the same candidates), plus a
confidence head trained to say whether that error is below 0.005 of the
stencil's range; in the solver, faces below the confidence threshold use the
eq. (28) weights.

Training: full-precision float32 master parameters, bf16 matrix-core
forward and backward (isweno_mlp_loss_grad), Adam (isweno_mlp_adam), all in
the library; this module only selects data and loops (none of the method's
arithmetic is done here).
"""
from __future__ import annotations

import math

import numpy as np

from . import isweno

# Optimal weights d_1..d_4 of the four candidate stencils (Sec. 3.3.1), per
# side, as the targets list them.
OPTIMAL_WEIGHTS = [0.4, 0.2, 0.3, 0.1]


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


def stratify(X, Y, share_nontrivial: float = 0.3, seed: int = 1707, limit: int | None = None):
    """Keeps every sample whose target weights differ from the optimal
    weights d_k by more than 0.05 on a side and enough of the others that
    the former are `share_nontrivial` of the set (or all of them if there
    are too few of the others)."""
    import torch
    d = torch.tensor(OPTIMAL_WEIGHTS * 2, dtype=Y.dtype, device=Y.device)
    dev = (Y - d).abs()
    nontriv = torch.maximum(dev[:, :4].amax(1), dev[:, 4:].amax(1)) > 0.05
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
    """The training loss on a set (from isweno_mlp_loss_grad, the labels of
    the confidence head formed by the kernel) and the share of samples the
    confidence head accepts at the threshold."""
    import torch
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    grad = torch.zeros(isweno.MLP_NPARAM, dtype=torch.float32, device="cuda")
    ctx.mlp_loss_grad(P, X, Y, None, loss, grad)
    out = torch.empty((X.shape[0], 9), dtype=torch.float32, device="cuda")
    ctx.mlp_forward(P, X, out)
    conf = torch.sigmoid(out[:, 8]) >= conf_threshold
    return {"loss": float(loss.item()), "frac_confident": float(conf.float().mean())}
