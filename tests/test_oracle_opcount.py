"""The oracle's operation counter against counts derived by hand.

oracle/opcount.cpp compiles the oracle on a counting number type: every
add, multiply, divide, square root and comparison is one operation; the
structural zeros and ones of L, R (eq. (11)) and of the flux directions
are free; a repeated operation on the same operands is counted once; a
value that no output or decision uses is not counted.  Each count below is
derived independently from the formulas the oracle follows, so a dropped
or doubled term in the counter (or a change of the oracle's arithmetic)
fails here.  The last tests tie the benchmark's per-unit constants to the
counter, on the states of the 2D shock-bubble and the 1D gas-liquid tube.
"""
import numpy as np
import pytest

import oracle
from paper_1707_00592_amd import workloads as wl

CLASSES = oracle.OP_CLASSES


def tot(c):
    return sum(c[k] for k in CLASSES)


# A smooth subsonic water state moving right: every test, no fallback,
# star speed S* > 0 so the left star state is the upwind one.
def _state(nt, scale=0.01, seed=0):
    rng = np.random.default_rng(seed)
    g = 1.0 / 3.4
    q = np.array([1000.0, 10.0] + [5.0] * nt + [1e5, g, 4.4 * 6e8 * g])
    return np.array([q * (1 + scale * rng.random(q.size)) for _ in range(6)])


def test_weno_is_counts():
    """Eqs. (19)-(28) on one stencil.
    Candidates (eq. (20)): 2+1, 2+1, 3+2, 3+2 -> 16.
    Indicators: beta1, beta2 2 each; beta3 12; beta4 11 (3c already made
    for beta3); beta12 9; tau5 15 (e-a, d-b, e+a, d+b, 2(d-b), 4(d+b), 6c
    and the two differences: 10, the squares 5) -> 51.
    Modified weights (eq. (28)): tau5/(beta12+eps) 2, alpha1,2 5 each,
    alpha3,4 4 each, sum 3, normalisation 4 -> 27.  Combination 4+3 = 7.
    Basic weights (eq. (21)): beta12 unused (-9), alpha 4 x 4, sum 3,
    normalisation 4.  Third order: only the 2-point stencils; beta1,
    beta2, beta12, tau5, and 2 normalisations."""
    v = np.random.default_rng(1).random(5)
    m = oracle.opcount_piece(0, 1, v)
    assert (tot(m), m["div"], m["sqrt"], m["cmp"]) == (16 + 51 + 27 + 7, 9, 0, 0)
    b = oracle.opcount_piece(0, 1, v, weights=oracle.W_BASIC)
    assert tot(b) == 16 + (51 - 9) + (16 + 3 + 4) + 7 and b["div"] == 8
    o3 = oracle.opcount_piece(0, 1, v, order=3)
    assert tot(o3) == 6 + (2 + 2 + 9 + 15) + (2 + 5 + 5 + 1 + 2) + 3


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_primitive_recovery_count(ndim):
    """Eq. (2): ndim velocity divisions, |u|^2 (ndim multiplies, ndim-1
    adds), p = (E - (rho/2)|u|^2 - Pi)/Gamma (2 multiplies, 2 subtractions,
    1 division)."""
    u = np.array([1.0] + [0.5] * ndim + [10.0, 2.5, 0.0])
    for d in range(ndim):
        c = oracle.opcount_prim(ndim, u, d)
        assert c == {"add": ndim - 1 + 2, "mul": ndim + 2, "div": ndim + 1, "sqrt": 0,
                     "cmp": 0}


def test_projection_count():
    """Averaged state: rho, p, Gamma, Pi (the velocities are not needed) 4 x
    (add, halve) = 8.  Eq. (11): c^2 5, c 1, rho c and rho c/2 2, 1/c^2 1
    (R's 1/(rho c) unused here) = 9.  Eq. (12) per cell: w1 = p/2 - (rho c/2)
    u (3), w2 = rho - p/c^2 (2), w_last = p/2 + (rho c/2) u (1, products
    shared), identity rows free: 6 x 6 = 36."""
    c = oracle.opcount_piece(1, 1, _state(1))
    assert tot(c) == 8 + 9 + 36 and c["sqrt"] == 1 and c["div"] == 2


def test_positivity_count():
    """rho > 0, Gamma > 0, (Gamma + 1) p + Pi > 0."""
    c = oracle.opcount_piece(3, 1, _state(1)[2])
    assert c == {"add": 2, "mul": 1, "div": 0, "sqrt": 0, "cmp": 3}


@pytest.mark.parametrize("nt", [0, 1, 2])
def test_hllc_count(nt):
    """Eqs. (14)-(18) with S* > 0: sound speeds 10 (+4 square roots of c and
    sqrt(rho)), averaged u 5, averaged c^2 12 (+1 root), S_L and S_R before
    clipping 4 (+2 comparisons), clipping 2 comparisons, S* 13 (rho_L u_L
    later reused as the momentum), left U and F 12 + 4 nt, S_k - S* tests 2
    (+2 comparisons), p_k 3, the left star flux 4 per component + 4 for the
    pressure terms, u* 2, sign of S* 1 comparison; the right star state and
    the right fluxes are not used (weights 0)."""
    q = _state(nt)
    c = oracle.opcount_piece(2, nt, np.concatenate([q[2], q[3]]))
    nc = 5 + nt
    arith = 10 + 5 + 12 + 4 + 13 + (12 + 4 * nt) + 2 + 3 + (4 * nc + 4) + 2
    assert (tot(c) - c["sqrt"] - c["cmp"], c["sqrt"], c["cmp"]) == (arith, 5, 7)
    assert tot(c) == 99 + 8 * nt
    # the mirrored face (S* < 0): the same arithmetic on the right star
    # state, and a second comparison for the sign of S*
    m = q[[3, 2]].copy()
    m[:, 1] = -m[:, 1]
    cm = oracle.opcount_piece(2, nt, m.ravel())
    assert tot(cm) - cm["cmp"] == tot(c) - c["cmp"] and cm["cmp"] == c["cmp"] + 1


def face_by_hand(nt):
    """Averaged state 8, face matrices 10 (R needed now), projection 36,
    (10 + nt) live reconstructions of 101 (the right transverse velocities
    feed only the unused right flux), less 5 operations shared by the left
    and right reconstruction of each of the five fields both sides use
    (q_i/2, q_{i+1}/2 and their sum, 2 q_i, 2 q_{i+1}), back-projection
    2 x 8, positivity 2 x 3 comparisons (the rest is shared with the sound
    speeds), HLLC."""
    return 8 + 10 + 36 + (10 + nt) * 101 - 5 * 5 + 16 + 6 + (99 + 8 * nt)


@pytest.mark.parametrize("nt", [0, 1, 2])
def test_face_count_is_the_sum_of_its_parts(nt):
    c, orders = oracle.opcount_face(nt, _state(nt))
    assert orders == (5, 5)
    assert tot(c) == face_by_hand(nt)
    c0, _ = oracle.opcount_face(nt, _state(nt), mood=False)
    assert tot(c) - tot(c0) == 6 and c["cmp"] - c0["cmp"] == 6


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_line_assembly_and_stage_update_counts(ndim):
    """Eqs. (5)-(6) per cell and axis: a flux difference and a scaling per
    component (2 nc), u* difference 1 and 3 per material source (7), plus nc
    to add the earlier axes' terms.  Runge-Kutta per cell and step: 2, 5, 5
    operations per component, less 2 products (Gamma/3 and Pi/3 of the last
    stage are also candidate terms of eq. (20) on those identity fields)."""
    p = wl.entropy_wave(8 if ndim < 3 else 5, ndim)
    g = oracle.make_grid(p.n, p.dx, p.bc_lo, p.bc_hi)
    o = oracle.make_opts()
    nc = 4 + ndim
    for d in range(ndim):
        total, faces, asm = oracle.opcount_line(p.U, g, o, d, 0)
        assert tot(asm) == p.n[d] * (2 * nc + 7 + (nc if d else 0)), (d, asm)
        assert tot(faces) == (p.n[d] + 1) * face_by_hand(ndim - 1)
    _, upd = oracle.opcount_step(p.U, g, o, 1e-4)
    assert tot(upd) == p.ncells * (12 * nc - 2)


def test_benchmark_constants_are_the_counted_ones():
    import bench
    for nd in (1, 2, 3):
        assert bench.FACE_OPS[nd] == face_by_hand(nd - 1)
        u = np.array([1.0] + [0.5] * nd + [10.0, 2.5, 0.0])
        assert bench.PRIM_OPS[nd] == tot(oracle.opcount_prim(nd, u))
        for d in range(nd):
            assert bench.axis_ops(nd, d) == 2 * (4 + nd) + 7 + ((4 + nd) if d else 0)
        assert bench.UPDATE_OPS_PER_STEP[nd] == 12 * (4 + nd) - 2
    # the tau5 = 0 form: candidates 16, tau5 15, combination 7, the test 1
    assert bench.SHORTCUT_SAVING_F64 == 101 - (16 + 15 + 7 + 1)
    # the FP32 flat return: four differences, three maxima, the test
    assert bench.SHORTCUT_SAVING_F32 == 101 - 8


def test_face_constant_is_a_lower_bound_on_benchmark_states():
    """On the 2D shock-bubble start (lines through the shock and the
    bubble) and the gas-liquid tube the mean count per face is at least the
    smooth-face constant and at most 15% above it: faces between states at
    rest have S* = 0 and pay for both star states of eq. (14), faces that
    fall back pay for a second reconstruction.  Throughput figures built on
    the constant therefore never overstate the work done."""
    import bench
    p = wl.shock_bubble_2d(256, 128)
    g = oracle.make_grid(p.n, p.dx, p.bc_lo, p.bc_hi)
    o = oracle.make_opts()
    nx, ny = p.n
    per = []
    for d, base in ((0, 64 * nx), (0, 60 * nx), (1, 128), (1, 230)):
        _, faces, _ = oracle.opcount_line(p.U, g, o, d, base)
        per.append(tot(faces) / (p.n[d] + 1))
    assert 1.0 <= min(per) / bench.FACE_OPS[2] and max(per) / bench.FACE_OPS[2] < 1.15, per
    q = wl.sod_gas_liquid(200)
    g1 = oracle.make_grid(q.n, q.dx, q.bc_lo, q.bc_hi)
    _, faces, _ = oracle.opcount_line(q.U, g1, o, 0, 0)
    r = tot(faces) / 201 / bench.FACE_OPS[1]
    assert 1.0 <= r < 1.15, r
