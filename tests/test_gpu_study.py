"""Basic against modified nonlinear weights on the GPU path (Sec. 3.3).

The modified weights of eq. (28) keep the formal order on smooth data with
critical points; the basic form of eq. (21) (q = 1, epsilon = 1e-40) falls
to about second order there.  The FP64 path equals the oracle bit for bit,
checked here on the smallest run of each form."""
import math

import numpy as np
import pytest

import oracle
from paper_1707_00592_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("weights", [0, 1])
def test_entropy_wave_run_matches_oracle_bitwise(lib, weights):
    import torch
    n, t_end = 40, 0.1
    steps = int(math.ceil(t_end / (0.5 * (1.0 / n) ** (5.0 / 3.0))))
    p = wl.entropy_wave(n, 1)
    ref, _, _, _ = oracle.run(p.U, oracle.make_grid(p.n, p.dx, 1, 1),
                              oracle.make_opts(weights=weights, mood=False),
                              nsteps=steps, dt=t_end / steps)
    ctx = lib.Context(0)
    g = lib.make_grid(p.n, p.dx, 1, 1)
    o = lib.make_opts(weights=weights, mood=False, cfl=0.0)
    U = torch.from_numpy(p.U.copy()).cuda()
    dt = torch.full((1,), t_end / steps, dtype=torch.float64, device="cuda")
    for _ in range(steps):
        ctx.rk3_step(U, g, o, dt)
    got = U.cpu().numpy()
    print(f"[study] weights={weights} n={n} steps={steps}", flush=True)
    assert np.array_equal(got, ref), np.abs(got - ref).max()


def test_modified_weights_keep_fifth_order_where_basic_weights_lose_it(lib):
    from paper_1707_00592_amd import studies
    ctx = lib.Context(0)
    res = studies.weights_study(ctx)
    for k, v in res.items():
        print(f"[study] {k}: L1 {np.array2string(np.array(v['l1']), precision=2)} "
              f"orders {v['orders']}", flush=True)
    for wave in ("sine", "pulse"):
        m, b = res[f"{wave}_modified"], res[f"{wave}_basic"]
        assert max(m["orders"][1:]) > 4.5, (wave, m)
        assert max(b["orders"]) < 3.0, (wave, b)
        assert m["l1"][-1] < 1e-2 * b["l1"][-1], (wave, m, b)
