"""The FP32 reconstruction/flux form against the FP64 oracle.

Not in the paper, so its bound is a measured one: projection, WENO-IS and
HLLC run in float32 (unit roundoff 6e-8) while primitive recovery, the
MOOD positivity test, the flux difference and the RK update stay float64.
Stated bounds (checked here): one RHS evaluation within 2e-4 relative L1 of
the oracle per component; a full shock-tube run within 1e-4 relative L1 in
rho and p and its error against the exact solution within 5 % of the FP64
path's (equal accuracy); every state admissible.
"""
import numpy as np
import pytest

import oracle
from paper_1707_00592_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _rel_l1(a, b):
    return np.abs(a - b).sum(axis=-1) / np.maximum(np.abs(b).sum(axis=-1), 1e-300)


@pytest.fixture(scope="module")
def ctx(lib):
    return lib.Context(0)


@pytest.mark.parametrize("shape", [(300,), (150, 70), (20, 18, 17), (70, 17, 33)])
def test_fp32_rhs_within_bound(lib, ctx, shape):
    p = wl.random_two_phase(shape, seed=11)
    og = oracle.make_grid(p.n, p.dx, p.bc_lo, p.bc_hi)
    ig = lib.make_grid(p.n, p.dx, p.bc_lo, p.bc_hi)
    ref, _ = oracle.rhs(p.U, og, oracle.make_opts())
    st = lib.new_stats()
    got = ctx.rhs(_dev(p.U), ig, lib.make_opts(precision=lib.FP32), stats=st).cpu().numpy()
    r = _rel_l1(got, ref)
    print(f"[fp32] rhs {shape}: rel L1 per comp {np.array2string(r, precision=2)}", flush=True)
    assert np.all(np.isfinite(got))
    assert r.max() < 2e-4
    assert lib.read_stats(st).status == 0


def test_fp32_shock_tube_equal_accuracy(lib, ctx):
    p = wl.sod_gas_liquid(200)
    og = oracle.make_grid(p.n, p.dx, 0, 0)
    ig = lib.make_grid(p.n, p.dx, 0, 0)
    ref, *_ = oracle.run(p.U, og, oracle.make_opts(mood=False), t_end=p.t_end)
    U = _dev(p.U)
    lib.Solver(ig, lib.make_opts(precision=lib.FP32, mood=False), ctx).run(U, t_end=p.t_end)
    got = U.cpu().numpy()
    pr_g = wl.cons_to_prim(got, 1); pr_r = wl.cons_to_prim(ref, 1)
    d_rho = _rel_l1(got[0], ref[0]); d_p = _rel_l1(pr_g["p"], pr_r["p"])
    W = oracle.exact_sample(p.extra["WL"], p.extra["WR"], (p.extra["x"] - 0.7) / p.t_end)
    e64 = np.abs(ref[0] - W[:, 0]).mean(); e32 = np.abs(got[0] - W[:, 0]).mean()
    print(f"[fp32] shock tube: rel L1 rho {d_rho:.2e} p {d_p:.2e}; L1 vs exact fp64 {e64:.4e} "
          f"fp32 {e32:.4e}", flush=True)
    assert d_rho < 1e-4 and d_p < 1e-4
    assert abs(e32 - e64) <= 0.05 * e64


def test_fp32_shock_bubble_stays_physical(lib, ctx):
    import torch
    p = wl.shock_bubble_2d(256, 128)
    ig = lib.make_grid(p.n, p.dx, 0, 0)
    U = _dev(p.U)
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    st = lib.new_stats()
    for _ in range(100):
        ctx.rk3_step(U, ig, lib.make_opts(precision=lib.FP32), dt, st)
    assert lib.read_stats(st).status == 0
    U64 = _dev(p.U)
    for _ in range(100):
        ctx.rk3_step(U64, ig, lib.make_opts(), dt)
    d = _rel_l1(U.cpu().numpy(), U64.cpu().numpy())
    print(f"[fp32] shock-bubble 256x128 x100: rel L1 vs fp64 {np.array2string(d, precision=2)}",
          flush=True)
    assert d[0] < 1e-3


def test_fp32_batch(lib, ctx):
    import torch
    b = wl.batch_riemann(64, seed=4, nmin=128, nmax=1024)
    ref, *_ = oracle.batch_step(b["U"], b["offsets"], b["dx"], oracle.make_opts(), nsteps=5)
    plan = ctx.batch_plan(b["offsets"], b["dx"])
    U = _dev(b["U"])
    dt = torch.zeros(64, dtype=torch.float64, device="cuda")
    plan.step(U, lib.make_opts(precision=lib.FP32), dt, nsteps=5)
    r = _rel_l1(U.cpu().numpy(), ref)
    print(f"[fp32] batch: rel L1 per comp {np.array2string(r, precision=2)}", flush=True)
    assert r[0] < 1e-4
