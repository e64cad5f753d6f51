"""Pins for the oracle's time step (reading R17: the Courant condition behind
the CFL number 0.5 of Secs. 5 and 6, dt = CFL / max over cells of
sum_d (|u_d| + c) / dx_d, taken from U^n once per step).

The expected values are built from the stiffened-gas sound speed in its
primitive form c^2 = gamma (p + Pinf) / rho (eq. (2) of the paper's model,
with gamma and Pinf as printed for water and air), not from the oracle's
(Gamma, Pi) form, so a mistake in the oracle's recovery of c, in the sum
over axes or in the max over cells shows up here:

* uniform water at rest and uniform moving air on grids with unequal
  dx, dy, dz: closed forms;
* the axis relation 1/dt_2D = 1/dt_x + 1/dt_y of a uniform state, with
  dt_x and dt_y from the oracle's own 1D runs;
* two cells moving along different axes: the max is over cells of the
  per-cell sum, which differs from summing per-axis maxima and from a max
  over axes.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1707_00592_amd import workloads as wl

WATER = (4.4, 6e8)
AIR = (1.4, 0.0)


def _c(rho, p, gamma, pinf):
    return math.sqrt(gamma * (p + pinf) / rho)


def _dt(U, n, dx, cfl=0.5):
    return oracle.cfl_dt(U, oracle.make_grid(n, dx), oracle.make_opts(cfl=cfl))


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_water_at_rest_closed_form(ndim):
    n = (5, 4, 3)[:ndim]
    dx = (0.1, 0.05, 0.02)[:ndim]
    N = int(np.prod(n))
    U = wl.prim_to_cons(np.full(N, 1000.0), [np.zeros(N)] * ndim, 1e5, *WATER)
    c = _c(1000.0, 1e5, *WATER)
    assert abs(c - 1624.9430759) < 1e-6  # sqrt(4.4 (1e5 + 6e8) / 1000)
    want = 0.5 / sum(c / h for h in dx)
    got = _dt(U, n, dx)
    assert abs(got - want) <= 1e-14 * want, (got, want)
    if ndim > 1:
        # a max over axes instead of the sum would give the finest axis alone
        assert abs(got - 0.5 / (c / min(dx))) > 1e-3 * want


@pytest.mark.parametrize("ndim", [2, 3])
def test_moving_air_closed_form(ndim):
    n = (4, 3, 2)[:ndim]
    dx = (0.3, 0.07, 0.011)[:ndim]
    vel = (30.0, -50.0, 70.0)[:ndim]
    N = int(np.prod(n))
    U = wl.prim_to_cons(np.full(N, 1.2), [np.full(N, v) for v in vel], 2e5, *AIR)
    c = _c(1.2, 2e5, *AIR)
    want = 0.5 / sum((abs(v) + c) / h for v, h in zip(vel, dx))
    got = _dt(U, n, dx)
    assert abs(got - want) <= 1e-14 * want, (got, want)
    # the CFL number scales dt linearly
    assert abs(_dt(U, n, dx, cfl=0.25) - 0.5 * got) <= 1e-15 * got


def test_axis_relation_against_1d_runs():
    """For a uniform state the per-cell sum over axes gives
    1/dt_2D = 1/dt_x + 1/dt_y, where dt_x and dt_y are the oracle's 1D time
    steps of the same state moving along that axis alone."""
    rho, p, (ux, uy) = 998.0, 3e7, (120.0, -45.0)
    dx, dy = 0.013, 0.004
    U1x = wl.prim_to_cons(np.full(6, rho), [np.full(6, ux)], p, *WATER)
    U1y = wl.prim_to_cons(np.full(6, rho), [np.full(6, uy)], p, *WATER)
    U2 = wl.prim_to_cons(np.full(12, rho), [np.full(12, ux), np.full(12, uy)], p, *WATER)
    tx = _dt(U1x, (6,), (dx,))
    ty = _dt(U1y, (6,), (dy,))
    t2 = _dt(U2, (4, 3), (dx, dy))
    assert abs(1.0 / t2 - (1.0 / tx + 1.0 / ty)) <= 1e-13 / t2


def test_max_is_over_cells_of_the_per_cell_sum():
    """Cell 0 moves fast along x, cell 1 fast along y (air, c = sqrt(1.4e5)).
    Per cell the sums are (|u|+c)/dx + c/dy and c/dx + (|v|+c)/dy; dt takes
    the larger one.  Summing per-axis maxima would count both fast speeds."""
    dx, dy = 0.01, 0.02
    rho, p = 1.0, 1e5
    u = np.array([900.0, 0.0])
    v = np.array([0.0, 900.0])
    U = wl.prim_to_cons(np.full(2, rho), [u, v], p, *AIR)
    c = _c(rho, p, *AIR)
    s0 = (900.0 + c) / dx + c / dy
    s1 = c / dx + (900.0 + c) / dy
    want = 0.5 / max(s0, s1)
    got = _dt(U, (2, 1), (dx, dy))
    assert abs(got - want) <= 1e-14 * want, (got, want)
    wrong = 0.5 / ((900.0 + c) / dx + (900.0 + c) / dy)
    assert abs(got - wrong) > 0.1 * want


def test_two_phase_field_takes_the_water_cell():
    """Water next to air at the same pressure: the water cell's sound speed
    (about 1625 m/s) sets dt, not the air cell's (374 m/s)."""
    U = wl.prim_to_cons(np.array([1000.0, 1.0]), [np.zeros(2)], 1e5,
                        np.array([WATER[0], AIR[0]]), np.array([WATER[1], AIR[1]]))
    want = 0.5 / (_c(1000.0, 1e5, *WATER) / 0.1)
    got = _dt(U, (2,), (0.1,))
    assert abs(got - want) <= 1e-14 * want
