"""The learned-weights form: bf16 matrix-core training and inference kernels
against the FP64 reference network of the oracle, and what the trained
network does in the solver.

Bounds (bf16 weights and activations carry 8 significant bits):
  * forward logits within 3e-2 * (1 + |z|) of the FP64 network evaluated on
    the same bf16-rounded parameters and inputs;
  * loss within 2 % and the gradient within 1e-2 (relative 2-norm, cosine
    similarity > 0.9999) of the FP64 gradient (loss: value error of the
    reconstructions the predicted weights give, plus the confidence term);
    the FP64 reference rounds nothing, while the kernels round the hidden
    activations and the back-propagated errors to bf16 (relative 2^-9 per
    value, through three layers forward and back);
  * every parameter block of the gradient within 1e-2 (relative 2-norm) of a
    reference that rounds to bf16 where the kernels do;
  * Adam and bf16 packing match their definitions to float32 rounding.
"""
import numpy as np
import pytest

import oracle
from paper_1707_00592_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _bf16(a):
    """Round float32 to bf16 (nearest even) and back, on the host."""
    u = np.asarray(a, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32)


@pytest.fixture(scope="module")
def ctx(lib):
    return lib.Context(0)


def _params(seed=0, scale=0.4):
    rs = np.random.default_rng(seed)
    return (rs.normal(scale=scale, size=oracle.MLP_NPARAM)).astype(np.float32)


def test_forward_matches_reference(lib, ctx):
    import torch
    rs = np.random.default_rng(1)
    P = _params(1)
    n = 1000  # several 32-row tiles and a ragged tail
    X = rs.uniform(0, 1, size=(n, 8)).astype(np.float32)
    out = torch.empty((n, 9), dtype=torch.float32, device="cuda")
    ctx.mlp_forward(_dev(P), _dev(X), out)
    got = out.cpu().numpy()
    ref = oracle.mlp_forward(_bf16(P).astype(np.float64), _bf16(X).astype(np.float64))
    err = np.abs(got - ref) / (1.0 + np.abs(ref))
    print(f"[mlp] forward max scaled err {err.max():.3e}", flush=True)
    assert err.max() < 3e-2


def test_solver_inference_matches_reference(lib, ctx):
    """The network as the stage kernel runs it (packed bf16 parameters,
    activations in registers, two 32-sample tiles per wavefront) against the
    FP64 network on the bf16-rounded parameters and inputs, over several
    waves and a ragged tail; and against the float32-master forward kernel."""
    import torch
    rs = np.random.default_rng(7)
    P = _params(7)
    n = 64 * 9 + 37
    X = rs.uniform(0, 1, size=(n, 8)).astype(np.float32)
    packed = torch.zeros(oracle.MLP_NPARAM, dtype=torch.int16, device="cuda")
    ctx.mlp_pack(_dev(P), packed)
    out = torch.empty((n, 9), dtype=torch.float32, device="cuda")
    ctx.mlp_infer(packed, _dev(X), out)
    got = out.cpu().numpy()
    ref = oracle.mlp_forward(_bf16(P).astype(np.float64), _bf16(X).astype(np.float64))
    err = np.abs(got - ref) / (1.0 + np.abs(ref))
    fwd = torch.empty((n, 9), dtype=torch.float32, device="cuda")
    ctx.mlp_forward(_dev(_bf16(P)), _dev(X), fwd)
    d = np.abs(got - fwd.cpu().numpy()) / (1.0 + np.abs(ref))
    print(f"[mlp] solver inference max scaled err {err.max():.3e}, vs forward kernel {d.max():.3e}",
          flush=True)
    assert err.max() < 3e-2
    assert d.max() < 1e-2


def test_loss_and_gradient_match_reference(lib, ctx):
    import torch
    rs = np.random.default_rng(2)
    P = _params(2, 0.3)
    n = 777
    X = rs.uniform(0, 1, size=(n, 8)).astype(np.float32)
    Y = rs.dirichlet(np.ones(4), size=(n, 2)).reshape(n, 8).astype(np.float32)
    Cc = (rs.random(n) < 0.5).astype(np.float32)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    grad = torch.zeros(oracle.MLP_NPARAM, dtype=torch.float32, device="cuda")
    ctx.mlp_loss_grad(_dev(P), _dev(X), _dev(Y), _dev(Cc), loss, grad)
    g = grad.cpu().numpy().astype(np.float64)
    lref, gref = oracle.mlp_loss_grad(_bf16(P).astype(np.float64), _bf16(X).astype(np.float64),
                                      Y.astype(np.float64), Cc.astype(np.float64))
    rel = np.linalg.norm(g - gref) / np.linalg.norm(gref)
    cos = g @ gref / (np.linalg.norm(g) * np.linalg.norm(gref))
    print(f"[mlp] loss {float(loss.item()):.6f} ref {lref:.6f}; grad rel {rel:.3e} cos {cos:.6f}",
          flush=True)
    assert abs(float(loss.item()) - lref) <= 0.02 * abs(lref)
    assert rel < 1e-2 and cos > 0.9999
    # deterministic: a second evaluation gives the same bits
    grad2 = torch.zeros_like(grad)
    ctx.mlp_loss_grad(_dev(P), _dev(X), _dev(Y), _dev(Cc), loss, grad2)
    assert torch.equal(grad, grad2)


def _rounded_reference_grad(P, X, Y, Cc):
    """The loss gradient with the kernels' bf16 roundings and float64
    everything else: inputs, weights, the hidden activations (after ReLU)
    and the back-propagated dz, dh2, dh1 rounded to bf16 where the kernels
    feed them to the matrix cores; biases, logits and the bias gradients
    unrounded.  Per-sample loss as isweno_mlp_loss_grad defines it (value
    error of the reconstructions over 0.01, squared, per side, plus the
    confidence cross-entropy)."""
    n = X.shape[0]
    W1 = _bf16(P[:256]).reshape(32, 8).astype(np.float64)
    b1 = P[256:288].astype(np.float64)
    W2 = _bf16(P[288:1312]).reshape(32, 32).astype(np.float64)
    b2 = P[1312:1344].astype(np.float64)
    W3 = _bf16(P[1344:1632]).reshape(9, 32).astype(np.float64)
    b3 = P[1632:1641].astype(np.float64)
    xb = _bf16(X).astype(np.float64)
    h1 = _bf16(np.maximum(xb @ W1.T + b1, 0.0)).astype(np.float64)
    h2 = _bf16(np.maximum(h1 @ W2.T + b2, 0.0)).astype(np.float64)
    z = h2 @ W3.T + b3
    x = X.astype(np.float64)

    def cands(a, b, c, d, e):
        return np.stack([0.5 * c + 0.5 * d, -0.5 * b + 1.5 * c,
                         c / 3 + 5 * d / 6 - e / 6, a / 3 - 7 * b / 6 + 11 * c / 6], axis=1)

    dz = np.zeros((n, 9))
    for h, cd in enumerate((cands(x[:, 0], x[:, 1], x[:, 2], x[:, 3], x[:, 4]),
                            cands(x[:, 5], x[:, 4], x[:, 3], x[:, 2], x[:, 1]))):
        zh = z[:, 4 * h:4 * h + 4]
        e = np.exp(zh - zh.max(axis=1, keepdims=True))
        w = e / e.sum(axis=1, keepdims=True)
        qh = (w * cd).sum(axis=1)
        qt = (Y[:, 4 * h:4 * h + 4].astype(np.float64) * cd).sum(axis=1)
        g = 2.0 * (qh - qt) / 0.01 ** 2 / n
        dz[:, 4 * h:4 * h + 4] = g[:, None] * w * (cd - qh[:, None])
    dz[:, 8] = (1.0 / (1.0 + np.exp(-z[:, 8])) - Cc) / n
    dzb = _bf16(dz).astype(np.float64)
    gW3 = dzb.T @ h2
    gb3 = dz.sum(axis=0)
    dh2 = (dzb @ W3) * (h2 > 0)
    gb2 = dh2.sum(axis=0)
    dh2b = _bf16(dh2).astype(np.float64)
    gW2 = dh2b.T @ h1
    dh1 = (dh2b @ W2) * (h1 > 0)
    gb1 = dh1.sum(axis=0)
    gW1 = _bf16(dh1).astype(np.float64).T @ xb
    return {"W1": gW1.ravel(), "b1": gb1, "W2": gW2.ravel(), "b2": gb2, "W3": gW3.ravel(),
            "b3": gb3}


BLOCKS = {"W1": slice(0, 256), "b1": slice(256, 288), "W2": slice(288, 1312),
          "b2": slice(1312, 1344), "W3": slice(1344, 1632), "b3": slice(1632, 1641)}


def test_gradient_blocks_match_the_rounded_reference(lib, ctx):
    """Every parameter block of the kernel gradient (W1, b1, W2, b2, W3, b3)
    within 1e-2 (relative 2-norm) of a reference that rounds to bf16 where
    the kernels do; what is left is float32 accumulation order and the odd
    bf16 tie that goes the other way."""
    import torch
    rs = np.random.default_rng(12)
    P = _params(12, 0.3)
    n = 777
    X = rs.uniform(0, 1, size=(n, 8)).astype(np.float32)
    Y = rs.dirichlet(np.ones(4), size=(n, 2)).reshape(n, 8).astype(np.float32)
    Cc = (rs.random(n) < 0.5).astype(np.float32)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    grad = torch.zeros(oracle.MLP_NPARAM, dtype=torch.float32, device="cuda")
    ctx.mlp_loss_grad(_dev(P), _dev(X), _dev(Y), _dev(Cc), loss, grad)
    g = grad.cpu().numpy().astype(np.float64)
    ref = _rounded_reference_grad(P, X, Y, Cc.astype(np.float64))
    for name, sl in BLOCKS.items():
        r = ref[name]
        rel = np.linalg.norm(g[sl] - r) / np.linalg.norm(r)
        print(f"[mlp] gradient block {name}: rel {rel:.2e}", flush=True)
        assert rel <= 1e-2, (name, rel)


def test_kernel_formed_confidence_targets(lib, ctx):
    """C = NULL: the label is 1 where the values both predicted heads
    reconstruct are within 0.005 of the target weights' values; equals
    passing those labels explicitly."""
    import torch
    from paper_1707_00592_amd import learned
    rs = np.random.default_rng(3)
    P = _params(3, 0.3)
    n = 300
    X = rs.uniform(0, 1, size=(n, 8)).astype(np.float32)
    out = torch.empty((n, 9), dtype=torch.float32, device="cuda")
    ctx.mlp_forward(_dev(P), _dev(X), out)
    z = out.cpu().numpy().astype(np.float64)
    soft = lambda a: np.exp(a - a.max(1, keepdims=True)) / np.exp(a - a.max(1, keepdims=True)).sum(1, keepdims=True)
    Yh = np.concatenate([soft(z[:, :4]), soft(z[:, 4:8])], axis=1)
    # the oracle's candidates of eq. (20) on the left stencils X[:, 0..4]
    cl = np.array([oracle.weno_candidates(x[:5]) for x in X.astype(np.float64)])
    # move 0.1 of weight between the first two left candidates on samples
    # where they differ by more than 0.2 (value error > 0.02), none elsewhere
    move = (rs.random(n) < 0.5) & (np.abs(cl[:, 0] - cl[:, 1]) > 0.2)
    Y = Yh + np.where(move, 0.1, 0.0)[:, None] * np.array([1, -1, 0, 0, 0, 0, 0, 0])
    Y = Y.astype(np.float32)
    C = (~move).astype(np.float32)
    assert 0 < C.sum() < n
    l1 = torch.zeros(1, device="cuda"); l2 = torch.zeros(1, device="cuda")
    g1 = torch.zeros(oracle.MLP_NPARAM, device="cuda"); g2 = torch.zeros_like(g1)
    ctx.mlp_loss_grad(_dev(P), _dev(X), _dev(Y), None, l1, g1)
    ctx.mlp_loss_grad(_dev(P), _dev(X), _dev(Y), _dev(C), l2, g2)
    assert float(l1.item()) == pytest.approx(float(l2.item()), rel=1e-5)
    np.testing.assert_allclose(g1.cpu().numpy(), g2.cpu().numpy(), rtol=1e-4, atol=1e-7)


def test_adam_step(lib, ctx):
    import torch
    rs = np.random.default_rng(4)
    P = rs.normal(size=oracle.MLP_NPARAM).astype(np.float32)
    G = rs.normal(size=oracle.MLP_NPARAM).astype(np.float32)
    M = rs.normal(size=oracle.MLP_NPARAM).astype(np.float32) * 0.1
    V = rs.uniform(0, 1, size=oracle.MLP_NPARAM).astype(np.float32) * 0.1
    p, m, v = _dev(P), _dev(M), _dev(V)
    ctx.mlp_adam(p, _dev(G), m, v, 3, 1e-3, 0.9, 0.999, 1e-8)
    b1, b2, lr, eps, t = 0.9, 0.999, 1e-3, 1e-8, 3
    m_ref = b1 * M + (1 - b1) * G
    v_ref = b2 * V + (1 - b2) * G * G
    p_ref = P - lr * (m_ref / (1 - b1 ** t)) / (np.sqrt(v_ref / (1 - b2 ** t)) + eps)
    np.testing.assert_allclose(m.cpu().numpy(), m_ref, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(v.cpu().numpy(), v_ref, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(p.cpu().numpy(), p_ref, rtol=1e-6, atol=1e-6)


def test_pack_rounds_to_nearest_even(lib, ctx):
    import torch
    P = _params(5)
    packed = torch.zeros(oracle.MLP_NPARAM, dtype=torch.int16, device="cuda")
    ctx.mlp_pack(_dev(P), packed)
    got = (packed.cpu().numpy().view(np.uint16).astype(np.uint32) << 16).view(np.float32)
    np.testing.assert_array_equal(got, _bf16(P))


def test_samples_match_reference_weights(lib, ctx):
    """Inputs and targets of isweno_mlp_samples against the oracle's own
    projection (L of eq. (11)) and weights (eq. (28)) on the same faces."""
    import torch
    p = wl.random_two_phase((40,), seed=6)
    ig = lib.make_grid(p.n, p.dx, 0, 0)
    n_rows = 41 * 5
    X = torch.zeros((n_rows, 8), dtype=torch.float32, device="cuda")
    Y = torch.zeros((n_rows, 8), dtype=torch.float32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    ctx.mlp_samples(_dev(p.U), ig, lib.make_opts(), X, Y, n_rows, 1, cnt)
    assert int(cnt.item()) == n_rows
    Xh, Yh = X.cpu().numpy(), Y.cpu().numpy()
    pr = wl.cons_to_prim(p.U, 1)
    q = np.stack([p.U[0], pr["vel"][0], pr["p"], p.U[3], p.U[4]], axis=1)
    ext = np.concatenate([np.repeat(q[:1], 3, 0), q, np.repeat(q[-1:], 3, 0)])
    for f in range(41):
        q6 = ext[f:f + 6]
        L, _ = oracle.eigen(0.5 * (q6[2] + q6[3]), 0)
        w = q6 @ L.T
        for m in range(5):
            row = f * 5 + m
            wl_ = oracle.weno_weights(w[:5, m])
            wr_ = oracle.weno_weights(w[5:0:-1, m])
            np.testing.assert_allclose(Yh[row], np.concatenate([wl_, wr_]), rtol=2e-6, atol=2e-7)
            lo, hi = w[:, m].min(), w[:, m].max()
            feat = (w[:, m] - lo) / (hi - lo) if hi - lo > 1e-30 else np.zeros(6)
            np.testing.assert_allclose(Xh[row, :6], feat, rtol=1e-5, atol=1e-6)


def test_samples_argument_errors(lib, ctx):
    """isweno_mlp_samples takes the solver's grid and option checks: a
    reflective end on an axis of fewer than 3 cells (whose ghost cells would
    fall outside the grid), an unused axis of more than one cell and an
    unknown weight form are refused before anything is launched."""
    import torch
    X = torch.zeros((64, 8), dtype=torch.float32, device="cuda")
    Y = torch.zeros((64, 8), dtype=torch.float32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    U = torch.zeros((5, 2), dtype=torch.float64, device="cuda")
    refl = lib.make_grid((2,), (0.1,), 2, 2)
    with pytest.raises(RuntimeError, match="invalid argument"):
        ctx.mlp_samples(U, refl, lib.make_opts(), X, Y, 64, 1, cnt)
    bad = lib.make_grid((2,), (0.1,))
    bad.n[1] = 3
    with pytest.raises(RuntimeError, match="invalid argument"):
        ctx.mlp_samples(U, bad, lib.make_opts(), X, Y, 64, 1, cnt)
    o = lib.make_opts()
    o.weights = 9
    with pytest.raises(RuntimeError, match="invalid argument"):
        ctx.mlp_samples(U, lib.make_grid((2,), (0.1,)), o, X, Y, 64, 1, cnt)


def test_training_and_learned_weights_in_the_solver(lib, ctx):
    """Train on faces from plain runs (gas-liquid shock tube and a small
    shock-droplet), then run the shock tube with the learned weights: the
    loss drops, the run stays physical, and its error against the exact
    solution is reported next to the plain FP32 path's.  Both runs use the
    MOOD cascade, the learned form's safety net behind its confidence
    fallback (without it a learned reconstruction at the water-air
    interface can turn a cell non-physical)."""
    import torch
    from paper_1707_00592_amd import learned
    opts64 = lib.make_opts()
    X, Y = learned.collect(ctx, [wl.sod_gas_liquid(200), wl.shock_droplet_3d(24, 3.0)],
                           opts64, steps=20, every=5, stride=3, max_rows=200000)
    Xs, Ys = learned.stratify(X, Y)
    P, hist = learned.train(ctx, Xs, Ys, steps=1500, batch=16384, lr=3e-3, log_every=500)
    print(f"[mlp] samples {Xs.shape[0]} loss history {hist}", flush=True)
    assert hist[-1][1] < 0.8 * hist[0][1]
    ev = learned.evaluate(ctx, P, Xs, Ys)
    print(f"[mlp] eval {ev}", flush=True)
    packed = torch.zeros(lib.MLP_NPARAM, dtype=torch.int16, device="cuda")
    ctx.mlp_pack(P, packed)
    # the same network before training (its initial parameters): what the
    # training gains
    packed0 = torch.zeros(lib.MLP_NPARAM, dtype=torch.int16, device="cuda")
    ctx.mlp_pack(_dev(learned.init_params(seed=1707)), packed0)
    p = wl.sod_gas_liquid(200)
    g = lib.make_grid(p.n, p.dx, 0, 0)
    og = oracle.make_grid(p.n, p.dx, 0, 0)
    ref, _, _, _ = oracle.run(p.U, og, oracle.make_opts(mood=True), t_end=p.t_end)
    W = oracle.exact_sample(p.extra["WL"], p.extra["WR"], (p.extra["x"] - 0.7) / p.t_end)
    res = {}
    for name, o in (("fp32", lib.make_opts(precision=lib.FP32, mood=True)),
                    ("mlp", lib.make_opts(precision=lib.FP32, weights=lib.W_MLP, mood=True,
                                          mlp_params=packed)),
                    ("untrained", lib.make_opts(precision=lib.FP32, weights=lib.W_MLP, mood=True,
                                                mlp_params=packed0))):
        U = _dev(p.U)
        st = lib.new_stats()
        _, _, k = lib.Solver(g, o, ctx).run(U, t_end=p.t_end, stats=st)
        s = lib.read_stats(st)
        got = U.cpu().numpy()
        # learned face-fields evaluated: 201 faces x 3 non-material fields x 3 stages per step
        evals = 201 * 3 * 3 * k
        res[name] = {"status": s.status, "o3": s.o3[0], "o1": s.o1[0],
                     "fallback_rate": s.mlp_fallback[0] / evals,
                     "l1_exact": np.abs(got[0] - W[:, 0]).mean() / 1000.0,
                     "l1_oracle": np.abs(got[0] - ref[0]).sum() / np.abs(ref[0]).sum()}
        print(f"[mlp] shock tube {name}: {res[name]}", flush=True)
        assert s.status == 0
    fp, ml, un = res["fp32"], res["mlp"], res["untrained"]
    print(f"[mlp] learned/plain error against the exact solution {ml['l1_exact'] / fp['l1_exact']:.3f}; "
          f"network weights used on {1 - ml['fallback_rate']:.3f} of the face-fields after "
          f"training, {1 - un['fallback_rate']:.3f} before", flush=True)
    # stated bounds of the learned form on this tube: within 2 % (relative
    # L1 of rho) of the FP64 oracle's run, within 30 % of the plain FP32
    # form's error against the exact solution, the network's own weights
    # kept on at least half of the face-fields; and training is what gets
    # it there (the untrained network falls back far more often)
    assert ml["l1_oracle"] < 2e-2
    assert ml["l1_exact"] < 1.3 * fp["l1_exact"]
    assert ml["fallback_rate"] < 0.5
    assert ml["fallback_rate"] < un["fallback_rate"]
