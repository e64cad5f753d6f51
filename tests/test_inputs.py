"""The synthetic inputs against the paper's tables and the shock relations.

Each post-shock state the paper prints is compared with the Rankine-
Hugoniot state of the stated shock strength, to the discrepancy the
printed values themselves carry (they are used as printed), so that a
transcription slip in the generators fails here.  Geometry: the cylinders
hold the expected number of cells.
"""
import math

import numpy as np
import pytest

from paper_1707_00592_amd import workloads as wl


def _rel(a, b):
    return abs(a - b) / abs(b)


def test_eq38_shock_droplet_states():
    """Eq. (38): a Mach 2 shock into air (1.2e-3, 0, 1, 1.4): density and
    pressure exactly the normal-shock values; the printed velocity 44.59 is
    4.4% above the shock's 42.70."""
    rho1, u1, p1, _ = wl.ideal_shock_from_mach(1.2e-3, 1.0, 1.4, 2.0)
    assert _rel(3.2e-3, rho1) < 1e-12 and _rel(4.5, p1) < 1e-12
    assert 0.04 < _rel(44.59, u1) < 0.05
    p = wl.shock_droplet_1d(400)
    x = p.extra["x"]
    rho = p.U[0]
    assert np.all(rho[x < 0.016] == 3.2e-3) and np.all(rho[(x > 0.0176) & (x < 0.0224)] == 1.0)
    assert p.n == (400,) and p.dx == (1e-4,)


def test_table1_post_shock_air():
    """Table 1: Ms = 1.22 into air (1.4, 0, 1e5, 1.4): the printed density
    1.927 and pressure 0.157 MPa are the normal-shock values to the printed
    digits; the printed speed 114.42 m/s is 8.5% above the shock's 105.5."""
    rho1, u1, p1, _ = wl.ideal_shock_from_mach(1.4, 1e5, 1.4, 1.22)
    assert _rel(1.927, rho1) < 1e-3 and _rel(1.57e5, p1) < 1e-3
    assert 0.08 < _rel(114.42, u1) < 0.09


def test_table2_post_shock_states():
    """Table 2: the Ms = 2 air shock (3.2, -434, 0.456 MPa; normal-shock
    values 3.2, 427.0, 0.45 MPa) and the 1 GPa water shock (1219.9, -424.55;
    stiffened-gas values with gamma 7, Pinf 0.331 GPa: 1188.0, 397.8)."""
    rho1, u1, p1, _ = wl.ideal_shock_from_mach(1.2, 1e5, 1.4, 2.0)
    assert _rel(3.2, rho1) < 1e-12
    assert _rel(4.56e5, p1) < 0.02 and _rel(434.0, u1) < 0.02
    rho1, u1, _ = wl.sg_shock_from_pressure(1000.0, 1e5, 7.0, 3.31e8, 1e9)
    assert 0.02 < _rel(1219.9, rho1) < 0.03 and 0.06 < _rel(424.55, u1) < 0.07


@pytest.mark.parametrize("gas,rho_in,gamma", [("R22", 4.415, 1.249), ("He", 0.255, 1.648)])
def test_gas_cylinder_layout(gas, rho_in, gamma):
    """Sec. 6.1 figure: 267 x 89 mm, 50 mm cylinder centred at (178, 44.5)
    mm, shock at 203 mm (post-shock air moving left), walls top and
    bottom."""
    p = wl.shock_gas_cylinder_2d(gas, 600, 200)
    nx, ny = p.n
    assert p.bc_lo == (0, 2) and p.bc_hi == (0, 2)
    assert math.isclose(p.dx[0], 0.267 / 600) and math.isclose(p.dx[1], 0.089 / 200)
    rho = p.U[0].reshape(ny, nx)
    G = p.U[4].reshape(ny, nx)
    inside = np.isclose(rho, rho_in)
    area = inside.sum() * p.dx[0] * p.dx[1]
    assert _rel(area, math.pi * 0.025 ** 2) < 0.01
    assert np.allclose(G[inside], 1.0 / (gamma - 1.0))
    mom = p.U[1].reshape(ny, nx)
    x = wl.cell_centres(nx, 0.0, 0.267)
    assert np.all(mom[:, x > 0.2035] < 0) and np.all(mom[:, x < 0.15] == 0)
    assert np.array_equal(rho, rho[::-1])        # symmetric about the axis


@pytest.mark.parametrize("case", ["droplet", "bubble"])
def test_air_water_layout(case):
    """Sec. 6.2 figure: 20 x 20 mm, 8 mm cylinder at (12, 10) mm, shock at
    16 mm, zero-gradient boundaries."""
    p = wl.air_water_2d(case, 400)
    nx, ny = p.n
    rho = p.U[0].reshape(ny, nx)
    inside = np.isclose(rho, 1000.0 if case == "droplet" else 1.0)
    assert _rel(inside.sum() * p.dx[0] * p.dx[1], math.pi * 0.004 ** 2) < 0.01
    assert p.bc_lo == (0, 0) and p.bc_hi == (0, 0)
