"""Pins for the oracle's WENO-IS reconstruction (paper Sec. 3.3).

Each check compares the oracle against something other than its own
formulas: exact polynomial reconstruction from cell averages (brute force
with rationals), the Jiang-Shu definition of the smoothness indicators as
integrals of squared derivatives, the paper's Taylor expansion (26),
stated properties (5th order on smooth data, 3rd order with d3 = d4 = 0,
the choice of a smooth 2-point stencil across close discontinuities) and
invariances.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle

# ---------------------------------------------------------------- helpers
def _solve(A, b):
    """Exact Gaussian elimination over Fractions."""
    n = len(b)
    M = [list(map(Fr, row)) + [Fr(v)] for row, v in zip(A, b)]
    for c in range(n):
        piv = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c] / M[c][c]
                M[r] = [x - f * y for x, y in zip(M[r], M[c])]
    return [M[r][n] / M[r][r] for r in range(n)]


def _cell_avg_monomial(j, m):
    """Average of x^m over the unit cell centred at integer j."""
    return (Fr(2 * j + 1, 2) ** (m + 1) - Fr(2 * j - 1, 2) ** (m + 1)) / (m + 1)


def fit_poly(cells, avgs):
    """Coefficients of the polynomial of degree len(cells)-1 whose unit-cell
    averages over `cells` equal `avgs`."""
    k = len(cells)
    A = [[_cell_avg_monomial(j, m) for m in range(k)] for j in cells]
    return _solve(A, avgs)


def poly_eval(c, x):
    return sum(ci * Fr(x) ** i for i, ci in enumerate(c))


def poly_deriv(c):
    return [i * c[i] for i in range(1, len(c))]


def poly_mul(a, b):
    out = [Fr(0)] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            out[i + j] += x * y
    return out


def poly_int(c, lo, hi):
    return sum(ci * (Fr(hi) ** (i + 1) - Fr(lo) ** (i + 1)) / (i + 1) for i, ci in enumerate(c))


def js_indicator(cells, avgs):
    """Jiang-Shu smoothness indicator on cell i = 0 (unit spacing): sum over
    l >= 1 of the integral over the cell of the squared l-th derivative of
    the reconstruction polynomial."""
    c = fit_poly(cells, avgs)
    beta = Fr(0)
    d = c
    for _ in range(len(cells) - 1):
        d = poly_deriv(d)
        beta += poly_int(poly_mul(d, d), Fr(-1, 2), Fr(1, 2))
    return beta


# stencil positions relative to cell i of the four candidates (Fig. 1)
STENCILS = {0: [0, 1], 1: [-1, 0], 2: [0, 1, 2], 3: [-2, -1, 0]}
FULL = [-2, -1, 0, 1, 2]


def _rand_int_stencil(rs, lo=-20, hi=20):
    return [int(v) for v in rs.integers(lo, hi, size=5)]


# ---------------------------------------------------------------- candidates
def test_candidates_are_polynomial_reconstructions():
    """Each candidate of eq. (20) is the face value x_{i+1/2} of the
    polynomial matching the cell averages of its stencil (Fig. 1).  This
    also settles the sign of the first candidate (printed with a minus)."""
    rs = np.random.default_rng(1)
    for _ in range(50):
        v = _rand_int_stencil(rs)
        cand = oracle.weno_candidates(v)
        for k, cells in STENCILS.items():
            exact = poly_eval(fit_poly(cells, [v[j + 2] for j in cells]), Fr(1, 2))
            assert cand[k] == pytest.approx(float(exact), rel=1e-14, abs=1e-12)


def test_linear_weights_give_fifth_order_upwind_scheme():
    """sum_k d_k q^(k) is the face value of the quartic through all five
    cell averages (the classical 5th-order scheme).  Rational check of the
    optimal weights d_k = (4, 2, 3, 1)/10 together with the candidates."""
    d = [Fr(4, 10), Fr(2, 10), Fr(3, 10), Fr(1, 10)]
    rs = np.random.default_rng(2)
    for _ in range(20):
        v = [Fr(int(x)) for x in rs.integers(-50, 50, size=5)]
        full = poly_eval(fit_poly(FULL, v), Fr(1, 2))
        comb = Fr(0)
        for k, cells in STENCILS.items():
            comb += d[k] * poly_eval(fit_poly(cells, [v[j + 2] for j in cells]), Fr(1, 2))
        assert comb == full


@pytest.mark.parametrize("weights", [oracle.W_MODIFIED, oracle.W_BASIC])
def test_tau5_zero_reproduces_linear_scheme(weights):
    """On quadratic data tau5 vanishes, the weights equal d_k and the
    oracle's reconstruction equals the exact face value (the 5th-order
    scheme is exact for quadratics)."""
    rs = np.random.default_rng(3)
    for _ in range(50):
        a2, a1, a0 = (int(x) for x in rs.integers(-9, 10, size=3))
        # scaled by 12 so that every cell average is an exact integer
        avgs = [12 * (a2 * _cell_avg_monomial(j, 2) + a1 * _cell_avg_monomial(j, 1) + a0)
                for j in FULL]
        v = [float(x) for x in avgs]
        assert oracle.weno_indicators(v)[5] == 0.0
        w = oracle.weno_weights(v, weights)
        np.testing.assert_allclose(w, [0.4, 0.2, 0.3, 0.1], rtol=1e-15)
        exact = 12 * (a2 * Fr(1, 4) + a1 * Fr(1, 2) + a0)
        assert oracle.weno_is(v, weights) == pytest.approx(float(exact), rel=1e-14, abs=1e-12)


def test_order3_with_linear_weights_is_third_order_scheme():
    """With d3 = d4 = 0 (Sec. 3.3.1) and tau5 = 0 the remaining weights are
    (2/3, 1/3): the 3rd-order reconstruction on {i-1, i, i+1}, exact for
    quadratics."""
    for (a2, a1, a0) in [(1, 0, 0), (3, -2, 5), (-4, 7, 1)]:
        avgs = [12 * (a2 * _cell_avg_monomial(j, 2) + a1 * _cell_avg_monomial(j, 1) + a0)
                for j in FULL]
        v = [float(x) for x in avgs]
        w = oracle.weno_weights(v, oracle.W_MODIFIED, order=3)
        np.testing.assert_allclose(w, [2 / 3, 1 / 3, 0, 0], rtol=1e-15, atol=0)
        central = poly_eval(fit_poly([-1, 0, 1], avgs[1:4]), Fr(1, 2))
        assert oracle.weno_is(v, order=3) == pytest.approx(float(central), rel=1e-14, abs=1e-12)


# ---------------------------------------------------------------- indicators
def test_indicators_match_jiang_shu_definition():
    """beta_1, beta_2 (2-point) and beta_3, beta_4, beta_12 (3-point) equal
    the integral of the squared derivatives of their reconstruction
    polynomials over cell i (eq. (24) and the beta_12 formula of Sec. 3.3.2,
    whose stencil is {i-1, i, i+1})."""
    rs = np.random.default_rng(4)
    for _ in range(40):
        v = _rand_int_stencil(rs)
        ind = oracle.weno_indicators(v)
        stencils = [STENCILS[0], STENCILS[1], STENCILS[2], STENCILS[3], [-1, 0, 1]]
        for k, cells in enumerate(stencils):
            ref = js_indicator(cells, [v[j + 2] for j in cells])
            assert ind[k] == pytest.approx(float(ref), rel=1e-14, abs=1e-12)


def test_tau5_leading_terms_match_taylor_expansion():
    """Eq. (26): tau5 = (q''')^2 dx^6 + 13/12 (q'''')^2 dx^8 + ...; exactly
    so for a pure cubic and for a pure even quartic (unit spacing)."""
    for s in [1, 2, -3]:
        cub = [float(s * (_cell_avg_monomial(j, 3))) for j in FULL]
        assert oracle.weno_indicators(cub)[5] == pytest.approx((6.0 * s) ** 2, rel=1e-14)
        qua = [float(s * (_cell_avg_monomial(j, 4))) for j in FULL]
        assert oracle.weno_indicators(qua)[5] == pytest.approx(13.0 / 12.0 * (24.0 * s) ** 2,
                                                               rel=1e-14)


def test_tau5_is_exactly_zero_on_equal_values_and_mirror_invariant():
    """Eq. (25) in floating point, formed with mirror points paired: any
    stencil of five equal finite values gives tau5 = 0 exactly (so the
    weights are exactly d_k, eqs. (21) and (28)), and a stencil and its
    mirror image give the same bits.  Pins the evaluation order: the
    left-to-right sum e - 4d + 6c - 4b + a leaves a rounding residue for
    most values (3c and 6c are not exact)."""
    rs = np.random.default_rng(11)
    vals = np.concatenate([rs.uniform(-1e9, 1e9, 300), rs.normal(size=300),
                           [1.0 / 3.4, 4.4 * 6e8 / 3.4, 1e-300, 1e300, -0.0]])
    residue = 0
    for c in vals:
        assert oracle.weno_indicators([c] * 5)[5] == 0.0, c
        assert list(oracle.weno_weights([c] * 5)) == [0.4 / 1.0000000000000002,
                                                      0.2 / 1.0000000000000002,
                                                      0.3 / 1.0000000000000002,
                                                      0.1 / 1.0000000000000002]
        t2 = c - 4.0 * c + 6.0 * c - 4.0 * c + c
        residue += t2 != 0.0
    assert residue > 100
    for _ in range(200):
        v = list(rs.normal(size=5) * 10.0 ** rs.integers(-5, 6))
        assert oracle.weno_indicators(v)[5] == oracle.weno_indicators(v[::-1])[5]


def test_indicators_scale_quadratically_and_ignore_constants():
    rs = np.random.default_rng(5)
    v = rs.normal(size=5)
    base = oracle.weno_indicators(v)
    np.testing.assert_allclose(oracle.weno_indicators(4.0 * v), 16.0 * base, rtol=1e-14)
    np.testing.assert_allclose(oracle.weno_indicators(v + 1e3), base, rtol=1e-8, atol=1e-9)


# ---------------------------------------------------------------- weights
def _isolate(smooth_k, rs, jump=1e6):
    """Stencil where only candidate stencil `smooth_k` (and, for the 3-point
    ones, the 2-point stencil inside it) is free of jumps."""
    base = rs.uniform(1, 2)
    slope = rs.uniform(-1, 1)
    lin = [base + slope * j for j in FULL]
    v = list(lin)
    if smooth_k == 0:      # S1 = {i, i+1}: jumps between i-1|i and i+1|i+2
        v[0] += jump; v[1] += jump; v[4] -= jump
    elif smooth_k == 1:    # S2 = {i-1, i}: jumps between i-2|i-1 and i|i+1
        v[0] -= jump; v[3] += jump; v[4] += jump
    elif smooth_k == 2:    # S3 = {i, i+1, i+2}: jump between i-1|i
        v[0] += jump; v[1] += jump
    else:                  # S4 = {i-2, i-1, i}: jump between i|i+1
        v[3] += jump; v[4] += jump
    face = base + slope * 0.5
    return v, face


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_smooth_stencil_is_selected_across_close_discontinuities(k):
    """Sec. 3.3.1: the reconstruction picks a smooth (2-point) stencil when
    every 3-point stencil is crossed by a discontinuity, and a smooth
    3-point stencil when one exists; the value then is the face value of
    the (linear) data on that stencil."""
    # The weights of the stencils crossed by a jump J scale as 1/J^2 and
    # their candidates as J, so the deviation from the smooth stencil's
    # value must shrink like 1/J.
    for weights in (oracle.W_MODIFIED, oracle.W_BASIC):
        for J in (1e4, 1e6, 1e8):
            rs = np.random.default_rng(10 + k)
            v, face = _isolate(k, rs, jump=J)
            assert abs(oracle.weno_is(v, weights) - face) < 10.0 / J
            w = oracle.weno_weights(v, weights)
            if k in (0, 1):
                assert w[k] > 1 - 10.0 / J


def _recon_error(f, F, N, x0=0.0, weights=oracle.W_MODIFIED, order=5):
    """Max error of the left face reconstruction at x0 + h/2 from exact cell
    averages of f (antiderivative F) on cells of size h = 1/N around x0."""
    h = 1.0 / N
    js = np.arange(-2, 3)
    avg = (F(x0 + (js + 0.5) * h) - F(x0 + (js - 0.5) * h)) / h
    return abs(oracle.weno_is(avg, weights, order=order) - f(x0 + 0.5 * h))


def _order(errs, Ns):
    return [np.log(errs[i] / errs[i + 1]) / np.log(Ns[i + 1] / Ns[i]) for i in range(len(Ns) - 1)]


@pytest.mark.parametrize("weights", [oracle.W_MODIFIED, oracle.W_BASIC])
def test_fifth_order_on_smooth_data(weights):
    """Eq. (27) and the convergence claims of Sec. 4: 5th order away from
    critical points (sampled at several phases)."""
    Ns = [40, 80, 160, 320]
    for phase in [0.3, 1.1, 2.0]:
        f = lambda x: np.sin(2 * np.pi * x + phase)
        F = lambda x: -np.cos(2 * np.pi * x + phase) / (2 * np.pi)
        errs = [_recon_error(f, F, N, 0.0, weights) for N in Ns]
        assert min(_order(errs, Ns)[1:]) > 4.6, errs


def test_modified_weights_keep_fifth_order_at_critical_point():
    """Sec. 3.3.2: the modification keeps 5th order near critical points
    (f' = 0 at the stencil centre)."""
    Ns = [40, 80, 160, 320]
    f = lambda x: np.cos(2 * np.pi * x)
    F = lambda x: np.sin(2 * np.pi * x) / (2 * np.pi)
    errs = [_recon_error(f, F, N, 0.0, oracle.W_MODIFIED) for N in Ns]
    assert min(_order(errs, Ns)[1:]) > 4.5, errs


def test_order3_variant_is_third_order():
    """d3 = d4 = 0 degenerates to a 3rd-order reconstruction (Sec. 3.3.1)."""
    Ns = [40, 80, 160, 320]
    f = lambda x: np.sin(2 * np.pi * x + 0.7)
    F = lambda x: -np.cos(2 * np.pi * x + 0.7) / (2 * np.pi)
    errs = [_recon_error(f, F, N, 0.0, oracle.W_MODIFIED, order=3) for N in Ns]
    o = _order(errs, Ns)
    assert 2.6 < min(o[1:]) and max(o[1:]) < 3.4, o


def test_weights_are_a_partition_of_unity_and_nonnegative():
    rs = np.random.default_rng(7)
    for _ in range(200):
        v = rs.normal(size=5) * 10.0 ** rs.integers(-3, 9)
        for weights in (oracle.W_MODIFIED, oracle.W_BASIC):
            w = oracle.weno_weights(v, weights)
            assert np.all(w >= 0)
            assert abs(w.sum() - 1.0) < 1e-14


def test_reconstruction_is_scale_and_shift_equivariant():
    rs = np.random.default_rng(8)
    for _ in range(50):
        v = rs.normal(size=5)
        q = oracle.weno_is(v)
        assert oracle.weno_is(8.0 * v) == pytest.approx(8.0 * q, rel=1e-13, abs=1e-13)
        assert oracle.weno_is(v + 3.0) == pytest.approx(q + 3.0, rel=1e-12, abs=1e-12)
        assert oracle.weno_is(-v) == pytest.approx(-q, rel=1e-13, abs=1e-13)
