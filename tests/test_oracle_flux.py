"""Pins for the oracle's characteristic decomposition, HLLC flux and MOOD
cascade (paper Secs. 3.2, 3.2.1, 3.4).

The primitive-variable Jacobian is rebuilt here from the conservation laws
(eqs. (1)-(3) with the EOS (2)) by complex-step differentiation, not from
the printed matrix A; flux checks use the Euler flux definition, contact
and supersonic special cases and mirror symmetry.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle


def _cons(q, nt):
    """U(q) and F(q) (face order) from eqs. (1)-(3) and the EOS (2); the
    material rows are the flux part phi*u of eq. (3)."""
    rho, un = q[0], q[1]
    ut = list(q[2:2 + nt])
    p, G, P = q[2 + nt], q[3 + nt], q[4 + nt]
    ke = un * un
    for v in ut:
        ke = ke + v * v
    E = G * p + P + Fr(1, 2) * rho * ke if isinstance(rho, _Dual) else G * p + P + 0.5 * rho * ke
    U = [rho, rho * un] + [rho * v for v in ut] + [E, G, P]
    F = [rho * un, rho * un * un + p] + [rho * un * v for v in ut] + [(E + p) * un, G * un, P * un]
    if isinstance(rho, _Dual):
        return U, F
    return np.array(U), np.array(F)


class _Dual:
    """a + b*eps with eps^2 = 0, over exact rationals (forward-mode
    derivative of the polynomial maps U(q), F(q))."""
    def __init__(self, a, b=0):
        self.a, self.b = Fr(a), Fr(b)

    def _w(self, o):
        return o if isinstance(o, _Dual) else _Dual(o)

    def __add__(self, o):
        o = self._w(o); return _Dual(self.a + o.a, self.b + o.b)
    __radd__ = __add__

    def __sub__(self, o):
        o = self._w(o); return _Dual(self.a - o.a, self.b - o.b)

    def __rsub__(self, o):
        return self._w(o) - self

    def __mul__(self, o):
        o = self._w(o); return _Dual(self.a * o.a, self.a * o.b + self.b * o.a)
    __rmul__ = __mul__


def _solve_exact(A, B):
    n = len(A)
    M = [list(A[r]) + list(B[r]) for r in range(n)]
    for c in range(n):
        piv = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c] / M[c][c]
                M[r] = [x - f * y for x, y in zip(M[r], M[c])]
    return [[M[r][n + k] / M[r][r] for k in range(len(B[0]))] for r in range(n)]


def _jacobian_primitive(q, nt):
    """A in dq/dt + A dq/dx = 0, derived exactly as M^-1 (N - B) with
    M = dU/dq, N = dF/dq (dual numbers over rationals) and B the
    non-conservative source phi du/dx of eq. (3)."""
    nc = 5 + nt
    qf = [Fr(float(v)) for v in q]
    M = [[Fr(0)] * nc for _ in range(nc)]
    N = [[Fr(0)] * nc for _ in range(nc)]
    for k in range(nc):
        qd = [_Dual(v, 1 if i == k else 0) for i, v in enumerate(qf)]
        U, F = _cons(qd, nt)
        for r in range(nc):
            M[r][k] = U[r].b if isinstance(U[r], _Dual) else Fr(0)
            N[r][k] = F[r].b if isinstance(F[r], _Dual) else Fr(0)
    N[3 + nt][1] -= qf[3 + nt]
    N[4 + nt][1] -= qf[4 + nt]
    A = _solve_exact(M, N)
    return np.array([[float(x) for x in row] for row in A])


def _random_state(rs, nt, water=None):
    water = rs.random() < 0.5 if water is None else water
    g, pinf = (4.4, 6e8) if water else (1.4, 0.0)
    rho = (1000.0 if water else 1.0) * rs.uniform(0.5, 2.0)
    p = 10 ** rs.uniform(5, 9)
    vel = rs.uniform(-300, 300, size=1 + nt)
    G, P = 1 / (g - 1), g * pinf / (g - 1)
    return np.array([rho, *vel, p, G, P])


def _sound(q, nt):
    return np.sqrt(((q[3 + nt] + 1) * q[2 + nt] + q[4 + nt]) / (q[3 + nt] * q[0]))


@pytest.mark.parametrize("nt", [0, 1, 2])
def test_eigenvectors_diagonalise_the_primitive_jacobian(nt):
    """Eq. (11): R = L^-1 and L A R = diag(u-c, u, ..., u, u+c) (eq. (10)),
    with A taken from the governing equations rather than eq. (9)."""
    rs = np.random.default_rng(20 + nt)
    for _ in range(20):
        q = _random_state(rs, nt)
        L, R = oracle.eigen(q, nt)
        nc = 5 + nt
        np.testing.assert_allclose(L @ R, np.eye(nc), atol=1e-12)
        A = _jacobian_primitive(q, nt)
        D = L @ A @ R
        c = _sound(q, nt)
        lam = np.array([q[1] - c] + [q[1]] * (nc - 2) + [q[1] + c])
        # entrywise rounding bound of the triple product
        bound = 1e-12 * (np.abs(L) @ np.abs(A) @ np.abs(R)) + 1e-300
        np.testing.assert_array_less(np.abs(D - np.diag(lam)), bound)


@pytest.mark.parametrize("nt", [0, 1, 2])
def test_hllc_consistency(nt):
    """F_hat(q, q) = F(q) and u^HLLC = u."""
    rs = np.random.default_rng(30 + nt)
    for _ in range(50):
        q = _random_state(rs, nt)
        F, us = oracle.hllc(q, q, nt)
        _, Fex = _cons(q, nt)
        np.testing.assert_allclose(F, Fex, rtol=1e-12, atol=1e-12 * np.abs(Fex).max())
        assert us == pytest.approx(q[1], rel=1e-12, abs=1e-12)


@pytest.mark.parametrize("nt", [0, 1])
def test_hllc_stationary_contact(nt):
    """u = 0 and equal p across a water/air contact: zero mass, energy and
    material fluxes, momentum flux p, u^HLLC = 0 (the equilibrium property
    behind Sec. 5.1)."""
    rs = np.random.default_rng(40)
    for _ in range(20):
        p = 10 ** rs.uniform(5, 9)
        ql = _random_state(rs, nt, water=True); qr = _random_state(rs, nt, water=False)
        ql[1:2 + nt] = 0.0; qr[1:2 + nt] = 0.0
        ql[2 + nt] = p; qr[2 + nt] = p
        F, us = oracle.hllc(ql, qr, nt)
        expect = np.zeros(5 + nt); expect[1] = p
        np.testing.assert_allclose(F, expect, atol=1e-9 * p)
        assert abs(us) < 1e-12


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_hllc_moving_contact_is_upwind(sign):
    """Equal u and p across a material interface: the flux is the upwind
    state's physical flux (pressure and velocity equilibrium)."""
    rs = np.random.default_rng(41)
    for _ in range(20):
        u0 = sign * rs.uniform(1, 300); p = 10 ** rs.uniform(5, 9)
        ql = _random_state(rs, 0, water=True); qr = _random_state(rs, 0, water=False)
        ql[1] = qr[1] = u0; ql[2] = qr[2] = p
        F, us = oracle.hllc(ql, qr, 0)
        _, Fup = _cons(ql if sign > 0 else qr, 0)
        np.testing.assert_allclose(F, Fup, rtol=1e-11, atol=1e-11 * np.abs(Fup).max())
        assert us == pytest.approx(u0, rel=1e-12)


def test_hllc_supersonic_is_upwind():
    """All waves moving one way: S_l (or S_r) is clipped to 0 and the
    two-branch formula of eq. (14) returns the upwind physical flux."""
    rs = np.random.default_rng(42)
    for _ in range(20):
        ql = _random_state(rs, 1, water=False); qr = ql.copy()
        qr[0] *= rs.uniform(0.9, 1.1); qr[3] *= rs.uniform(0.9, 1.1)
        for s in (1.0, -1.0):
            a, b = ql.copy(), qr.copy()
            c = max(_sound(a, 1), _sound(b, 1))
            a[1] = b[1] = s * 3.0 * c
            F, _ = oracle.hllc(a, b, 1)
            _, Fup = _cons(a if s > 0 else b, 1)
            np.testing.assert_allclose(F, Fup, rtol=1e-12, atol=1e-12 * np.abs(Fup).max())


@pytest.mark.parametrize("nt", [0, 1])
def test_hllc_mirror_symmetry(nt):
    """Reflecting the problem (swap sides, negate normal velocity) negates
    the mass, transverse-momentum, energy and material fluxes and u^HLLC and
    keeps the normal-momentum flux."""
    rs = np.random.default_rng(43)
    for _ in range(50):
        ql = _random_state(rs, nt); qr = _random_state(rs, nt)
        F, us = oracle.hllc(ql, qr, nt)
        ml, mr = qr.copy(), ql.copy()
        ml[1] = -ml[1]; mr[1] = -mr[1]
        Fm, usm = oracle.hllc(ml, mr, nt)
        sign = -np.ones(5 + nt); sign[1] = 1.0
        np.testing.assert_allclose(Fm, sign * F, rtol=1e-10, atol=1e-10 * np.abs(F).max())
        assert usm == pytest.approx(-us, rel=1e-10, abs=1e-10 * (abs(us) + 1))


def test_hllc_pstar_equal_on_both_sides():
    """The star pressures of eq. (15) coincide: p + rho_k (S_k - u_k)(S* - u_k)
    is the same for k = l and k = r, since S* is defined by eq. (16)."""
    rs = np.random.default_rng(44)
    for _ in range(50):
        ql = _random_state(rs, 0); qr = _random_state(rs, 0)
        cl, cr = _sound(ql, 0), _sound(qr, 0)
        sl, sr = np.sqrt(ql[0]), np.sqrt(qr[0])
        ub = (sl * ql[1] + sr * qr[1]) / (sl + sr)
        cb = np.sqrt((sl * cl**2 + sr * cr**2) / (sl + sr)
                     + 0.5 * sl * sr / (sl + sr) ** 2 * (qr[1] - ql[1]) ** 2)
        Sl = min(ub - cb, ql[1] - cl, 0.0); Sr = max(ub + cb, qr[1] + cr, 0.0)
        F, us = oracle.hllc(ql, qr, 0)
        # recover S* from the flux's energy/momentum structure
        Ss = (qr[2] - ql[2] + ql[0] * ql[1] * (Sl - ql[1]) - qr[0] * qr[1] * (Sr - qr[1])) / \
             (ql[0] * (Sl - ql[1]) - qr[0] * (Sr - qr[1]))
        pl = ql[2] + ql[0] * (Sl - ql[1]) * (Ss - ql[1])
        pr = qr[2] + qr[0] * (Sr - qr[1]) * (Ss - qr[1])
        assert pl == pytest.approx(pr, rel=1e-9)
        # the mass flux of the upwind star state is rho*(S-u)/(S-S*) * S*
        k = ql if Ss > 0 else qr
        S = Sl if Ss > 0 else Sr
        if S != Ss:
            assert F[0] == pytest.approx(k[0] * (S - k[1]) / (S - Ss) * Ss, rel=1e-10,
                                         abs=1e-10 * abs(F[0]) + 1e-12)


# ------------------------------------------------------------------ face/MOOD
def _stencil(rs, nt, wild=False):
    q6 = np.array([_random_state(rs, nt) for _ in range(6)])
    if wild:
        # alternating water/air with large pressure and velocity jumps
        for j in range(6):
            water = (j + rs.integers(2)) % 2 == 0
            q6[j] = _random_state(rs, nt, water=water)
            q6[j, 1] = rs.uniform(-3000, 3000)
            q6[j, 2 + nt] = 10 ** rs.uniform(4, 9.5)
    return q6


def _back_project(q6, nt, order, side):
    nc = 5 + nt
    qbar = 0.5 * (q6[2] + q6[3])
    L, R = oracle.eigen(qbar, nt)
    w = q6 @ L.T
    wt = np.zeros(nc)
    for m in range(nc):
        v = w[:5, m] if side == 0 else w[5:0:-1, m]
        wt[m] = oracle.weno_is(v, order=order)
    return R @ wt


@pytest.mark.parametrize("nt", [0, 1])
def test_mood_cascade_outputs_are_admissible(nt):
    """Sec. 3.4: every state handed to HLLC with MOOD on is admissible; a
    side reported at order 3 failed the check at order 5, a side at order 1
    failed it at orders 5 and 3 and equals the cell state (eq. (32))."""
    rs = np.random.default_rng(50 + nt)
    on = oracle.make_opts(mood=True)
    seen = {5: 0, 3: 0, 1: 0}
    for _ in range(3000):
        q6 = _stencil(rs, nt, wild=True)
        if not all(oracle.pos(q, nt) for q in q6):
            continue
        ql, qr, orders, F, us = oracle.face(q6, nt, on)
        assert oracle.pos(ql, nt) and oracle.pos(qr, nt)
        assert np.all(np.isfinite(F)) and np.isfinite(us)
        for side, (q, o) in enumerate(zip((ql, qr), orders)):
            seen[o] += 1
            q5 = _back_project(q6, nt, 5, side)
            if o == 5:
                np.testing.assert_allclose(q, q5, rtol=1e-12, atol=1e-12 * np.abs(q5).max())
            else:
                assert not oracle.pos(q5, nt)
                q3 = _back_project(q6, nt, 3, side)
                if o == 3:
                    np.testing.assert_allclose(q, q3, rtol=1e-12, atol=1e-12 * np.abs(q3).max())
                else:
                    assert not oracle.pos(q3, nt)
                    np.testing.assert_array_equal(q, q6[2 + side])
    assert seen[3] > 0 and seen[1] > 0 and seen[5] > 0, seen


def test_mood_off_keeps_fifth_order_state():
    rs = np.random.default_rng(60)
    off = oracle.make_opts(mood=False)
    for _ in range(100):
        q6 = _stencil(rs, 1, wild=True)
        ql, qr, orders, F, us = oracle.face(q6, 1, off)
        assert orders == (5, 5)
        np.testing.assert_allclose(ql, _back_project(q6, 1, 5, 0), rtol=1e-12,
                                   atol=1e-12 * np.abs(ql).max())


def test_face_of_uniform_stencil_is_physical_flux():
    rs = np.random.default_rng(61)
    for nt in (0, 1, 2):
        q = _random_state(rs, nt)
        q6 = np.tile(q, (6, 1))
        ql, qr, orders, F, us = oracle.face(q6, nt)
        _, Fex = _cons(q, nt)
        np.testing.assert_allclose(ql, q, rtol=1e-12, atol=1e-12 * np.abs(q).max())
        np.testing.assert_allclose(F, Fex, rtol=1e-11, atol=1e-11 * np.abs(Fex).max())
