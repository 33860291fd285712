"""Pins of the oracle's flume diagnostics and flow-rate control (Section 3.1
drives the flow by a body force controlled to hold the bulk flow rate;
Section 3.2 defines the y-averaged solid fraction phi_b and the bed height
h_b where phi_b = 0.3).

* phi_b of one sphere sums to the number of cell centres inside it, counted
  here directly from the geometry;
* h_b: a linear phi_b profile crosses 0.3 exactly where the line does; a
  solid slab; no solid cells; a bed up to the top;
* bulk velocity of the initial state: u0 - g/2 (the stored momentum carries
  half of the force step);
* the controller drives a gravity-free film to its target bulk velocity, and
  the force it settles on is the one of the Nusselt film,
  U = g h^2 / (3 nu) for the parabolic profile (cell-averaged here).
"""
import numpy as np

from oracle import oracle as O
from paper_2301_10674_amd import inputs as I


def test_phi_b_counts_sphere_cells():
    nx, ny, nz = 24, 16, 20
    o = O.OracleLattice((nx, ny, nz), 1.5, fill=np.ones((nz, ny, nx)))
    c, r = np.array([11.3, 7.6, 9.2]), 4.7
    o.set_particles(c[None, :], [r])
    phi, h = O.bed_profile(o.read(O.F_TYPE))
    z, y, x = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5, np.arange(nx) + 0.5, indexing="ij")
    inside = (x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2 <= r * r
    assert phi.shape == (nz, nx)
    assert np.isclose(phi.sum() * ny, inside.sum(), rtol=0, atol=1e-9)
    assert np.allclose(phi * ny, inside.sum(axis=1), rtol=0, atol=1e-12)


def test_h_b_crossings():
    nz, ny, nx = 12, 20, 4
    t = np.full((nz, ny, nx), O.LIQUID, dtype=np.uint8)
    # column 0: phi_b(z) = 0.95 - 0.1 z (cell index z), a line through the
    # cell centres z + 1/2 that crosses 0.3 at 7.0
    for k in range(nz):
        n = int(round(ny * max(0.95 - 0.1 * k, 0.0)))
        t[k, :n, 0] = O.SOLID
    # column 1: solid slab of 5 cells -> between centres 4.5 (1) and 5.5 (0)
    t[:5, :, 1] = O.SOLID
    # column 2: no solid cells; column 3: solid to the top
    t[:, :, 3] = O.SOLID
    phi, h = O.bed_profile(t)
    assert abs(h[0] - 7.0) < 1e-12
    assert abs(h[1] - (4.5 + 0.7)) < 1e-12
    assert h[2] == 0.0
    assert h[3] == nz


def test_bulk_velocity_of_the_initial_state():
    nx, ny, nz = 6, 5, 9
    u0 = np.array([3e-3, -1e-3, 5e-4])
    g = np.array([2e-5, 0.0, -4e-5])
    vel = np.broadcast_to(u0[:, None, None, None], (3, nz, ny, nx)).copy()
    fill = np.ones((nz, ny, nx))
    fill[6:] = 0.0
    fill[6] = 0.4
    o = O.OracleLattice((nx, ny, nz), 1.3, accel=tuple(g), fill=fill, vel=vel)
    assert np.allclose(O.bulk_velocity(o), u0 - 0.5 * g, rtol=0, atol=1e-15)


def test_controller_reaches_the_nusselt_film_force():
    h, omega = 10.5, 1.0
    nu = (1.0 / omega - 0.5) / 3.0
    w = I.flat_film((3, 3, 19), h=h, omega=omega, gx=0.0)
    o = O.OracleLattice(w.shape, w.omega, accel=(0.0, 0.0, 0.0), fill=w.fill)
    # liquid cells 0..9, the interface cell 10 with fill 1/2, stress-free
    # surface at its outer face (hs = 11): U per unit force of the
    # parabolic profile, averaged over the cells like the bulk velocity
    hs = 11.0
    zc = np.arange(19) + 0.5
    wts = np.zeros(19)
    wts[:10] = 1.0
    wts[10] = 0.5
    K = (wts * zc * (2 * hs - zc) / (2 * nu)).sum() / wts.sum()
    target = 1e-3
    ctl = O.FlowController(target, 0.0, kp=1.0 / K, ki=0.2 / K, every=50)
    ax = ctl.run(o, 6000)
    assert abs(O.bulk_velocity(o)[0] / target - 1.0) < 1e-6
    assert abs(ax * K / target - 1.0) < 0.01
