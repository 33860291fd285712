"""Pins of the particle oracle (dem_oracle.c): rigid spheres with contacts,
lubrication, gravity and a hydrodynamic load, sub-stepped within a lattice
step (Section 2.2 names the model's parameters e_dry, T_c, nu_p, mu_p and
the lubrication corrections; the readings are the linear spring-dashpot,
Coulomb-capped tangential spring and Brenner's normal lubrication force).

Closed forms and invariants, none retyping the oracle's formulas:

* a free head-on collision (equal or unequal spheres, a sphere on the wall
  or on a fixed sphere) rebounds with the relative speed scaled by e_dry
  and lasts T_c: a damped oscillator on the overlap whose stiffness and
  damping follow from the effective mass;
* an oblique collision of spinning spheres conserves linear momentum and
  angular momentum about the origin (to rounding);
* a sphere sliding on the wall under gravity decelerates at mu g while it
  slides and ends rolling (angular momentum about the contact point is
  conserved: 5/7 of its initial speed for a point contact);
* two spheres (or a sphere and the wall) approaching inside the
  lubrication range follow the integral of m du = 6 pi mu R_eff^2 (1/s -
  1/s_c) ds, u(s) = u0 - 6 pi mu R_eff^2/m_eff (ln(s0/s) - (s0 - s)/s_c);
* a sphere sliding along the wall inside the lubrication range ends
  rolling (angular momentum about the gap's midpoint is conserved) and its
  slip decays at the rate the tangential coefficient 8 r/15 gives; two equal
  spheres sliding past each other at the rate of r/6;
* a constant hydrodynamic force and torque accelerate a sphere of mass
  rho_p 4/3 pi r^3 and moment of inertia 2/5 m r^2 uniformly;
* the bedload rate of Eq. (1) for spheres moving together, opposite pairs,
  fixed spheres and scaled velocities.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O

RHO = 2.5


def mass(r):
    return RHO * 4.0 / 3.0 * math.pi * r ** 3


def collide(centres, radii, vel, box=(200, 200, 200), fixed=None, steps=400, h=0.05, **kw):
    """run until the bodies separate; returns velocities after and the
    number of sub-steps in contact"""
    d = O.OracleDem(box, centres, radii, vel=vel, fixed=fixed, density=RHO, dt=h, substeps=1, **kw)
    inside = 0
    for _ in range(steps):
        d.step()
        x, v, w = d.state()
        if len(radii) == 2:
            gap = np.linalg.norm(x[1] - x[0]) - radii[0] - radii[1]
        else:
            gap = x[0, 2] - radii[0]
        inside += gap < 0
        if inside and gap > 0.5:
            break
    return v, inside * h


@pytest.mark.parametrize("r1,r2", [(5.0, 5.0), (4.0, 6.5)])
def test_head_on_restitution_and_duration(r1, r2):
    u = 0.02
    v, tc = collide([[100, 100, 100], [100, 100, 100 + r1 + r2 + 0.2]], [r1, r2],
                    [[0, 0, u], [0, 0, -u]], steps=2000)
    m1, m2 = mass(r1), mass(r2)
    # centre-of-mass velocity unchanged; relative velocity reversed and scaled by e
    assert abs(m1 * v[0, 2] + m2 * v[1, 2] - (m1 - m2) * u) < 1e-12 * m1 * u
    e = (v[1, 2] - v[0, 2]) / (2 * u)
    assert abs(e - 0.97) < 5e-4, e
    assert abs(tc - 40.0) <= 0.1, tc
    assert np.abs(v[:, :2]).max() == 0.0


def test_wall_and_fixed_partner_restitution():
    u = 0.02
    v, tc = collide([[50, 50, 5.1]], [5.0], [[0, 0, -u]], box=(100, 100, 100), steps=2000)
    assert abs(v[0, 2] / u - 0.97) < 5e-4 and abs(tc - 40.0) <= 0.1
    v, tc = collide([[50, 50, 40.0], [50, 50, 50.1]], [5.0, 5.0], [[0, 0, 0], [0, 0, -u]],
                    fixed=[1, 0], box=(100, 100, 100), steps=2000)
    assert v[0, 2] == 0.0
    assert abs(v[1, 2] / u - 0.97) < 5e-4 and abs(tc - 40.0) <= 0.1


def angular_momentum(x, v, w, r):
    m = np.array([mass(q) for q in r])
    inertia = 0.4 * m * np.asarray(r) ** 2
    return (np.cross(x, m[:, None] * v) + inertia[:, None] * w).sum(0), (m[:, None] * v).sum(0)


def test_oblique_spinning_collision_conserves_momenta():
    r = [5.0, 3.5]
    x0 = [[100, 100, 100], [108.0, 103.0, 101.0]]
    v0 = [[0.03, 0.01, 0.0], [-0.02, -0.01, 0.005]]
    w0 = [[0.0, 0.004, -0.003], [0.002, 0.0, 0.006]]
    d = O.OracleDem((200, 200, 200), x0, r, vel=v0, angvel=w0, density=RHO, dt=1.0, substeps=20,
                    friction=0.3)
    L0, P0 = angular_momentum(np.array(x0, float), np.array(v0), np.array(w0), r)
    touched = False
    for _ in range(150):
        d.step()
        x, v, w = d.state()
        touched |= np.linalg.norm(x[1] - x[0]) < 8.5
    assert touched
    L1, P1 = angular_momentum(x, v, w, r)
    assert np.abs(P1 - P0).max() < 1e-12 * np.abs(P0).max()
    assert np.abs(L1 - L0).max() < 1e-11 * np.abs(L0).max()
    # the spins changed: the tangential force acted
    assert np.abs(w - np.array(w0)).max() > 1e-4


def test_sliding_sphere_ends_rolling():
    """Angular momentum about the contact point is conserved (gravity, the
    normal force and the friction force have no lever about it), so the
    sphere ends rolling at v0 / (1 + I/(m l^2)), l the distance from its
    centre to the contact point -- 5/7 of v0 for a point contact, here with
    l = r - delta/2 for the resting overlap delta = m g / k_n."""
    r, g, mu, v0 = 5.0, 2e-3, 0.05, 0.1
    k_n = mass(r) * (math.pi ** 2 + math.log(0.97) ** 2) / 40.0 ** 2
    delta = mass(r) * g / k_n
    d = O.OracleDem((4000, 50, 50), [[20, 25, r - delta]], [r], vel=[[v0, 0, 0]], density=RHO,
                    accel=(0, 0, -g), friction=mu, dt=1.0, substeps=20)
    t_roll = 2 * v0 / (7 * mu * g)                  # sliding ends about here
    vs, ws = [], []
    for k in range(int(5 * t_roll)):
        d.step()
        x, v, w = d.state()
        vs.append(v[0, 0])
        ws.append(w[0, 1])
        assert abs(w[0, 0]) < 1e-12 and abs(w[0, 2]) < 1e-12
    vs, ws = np.array(vs), np.array(ws)
    # sliding phase: deceleration mu g
    k1, k2 = int(0.2 * t_roll), int(0.7 * t_roll)
    assert abs((vs[k1] - vs[k2]) / (k2 - k1) / (mu * g) - 1) < 1e-6
    # rolling phase (the tangential spring rings about it: time means)
    ell = r - delta / 2
    a, b = int(2 * t_roll), int(5 * t_roll)
    want = 1 / (1 + 0.4 * (r / ell) ** 2)
    assert abs(vs[a:b].mean() / v0 - want) < 2e-4, (vs[a:b].mean() / v0, want)
    assert abs((ws[a:b] * ell).mean() / vs[a:b].mean() - 1) < 2e-4


@pytest.mark.parametrize("wall", [False, True])
def test_lubrication_approach_matches_the_integral(wall):
    mu, sc, r, u0 = 0.01, 0.8, 5.0, 0.01
    s0, s1 = 0.7, 0.05
    h = 0.02
    if wall:
        d = O.OracleDem((100, 100, 100), [[50, 50, r + s0]], [r], vel=[[0, 0, -u0]], density=RHO,
                        viscosity=mu, lub_cut=sc, lub_min=1e-4, dt=h, substeps=1)
        reff, meff = r, mass(r)
    else:
        d = O.OracleDem((100, 100, 100), [[50, 50, 40], [50, 50, 40 + 2 * r + s0]], [r, r],
                        vel=[[0, 0, u0 / 2], [0, 0, -u0 / 2]], density=RHO, viscosity=mu,
                        lub_cut=sc, lub_min=1e-4, dt=h, substeps=1)
        reff, meff = r / 2, mass(r) / 2
    for _ in range(int(4 * (s0 - s1) / (u0 * h))):  # at least half the speed is kept
        d.step()
        x, v, w = d.state()
        s = x[0, 2] - r if wall else x[1, 2] - x[0, 2] - 2 * r
        u = -v[0, 2] if wall else v[0, 2] - v[1, 2]
        if s <= s1:
            break
    assert s <= s1, (s, u)
    want = u0 - 6 * math.pi * mu * reff ** 2 / meff * (math.log(s0 / s) - (s0 - s) / sc)
    assert want < 0.8 * u0                            # the correction matters
    assert abs(u - want) < 2e-3 * u0, (u, want)


def test_hydrodynamic_load_and_fixed_spheres():
    r = [4.0, 3.0]
    F = np.array([[1e-3, -2e-3, 5e-4, 1e-2, 0, -3e-2], [1, 1, 1, 1, 1, 1]], float)
    d = O.OracleDem((100, 100, 100), [[30, 30, 50], [70, 70, 50]], r, fixed=[0, 1], density=RHO,
                    dt=1.0, substeps=7)
    d.step(F, n=10)
    x, v, w = d.state()
    m = mass(r[0])
    assert np.allclose(v[0], F[0, :3] * 10 / m, rtol=1e-13, atol=0)
    assert np.allclose(w[0], F[0, 3:] * 10 / (0.4 * m * r[0] ** 2), rtol=1e-13, atol=0)
    assert np.array_equal(x[1], [70, 70, 50]) and not v[1].any() and not w[1].any()


def test_bedload_rate():
    """Eq. (1): q_b = sum_i u_x,i V_i / (Lx Ly).  Spheres moving together at
    u give u times their total volume over the bed area; a sphere moving
    against the stream cancels an equal one moving with it; fixed spheres
    (at rest) add nothing; the rate is linear in the velocities."""
    box = (60, 20, 40)
    r = np.array([2.0, 3.0, 2.0, 4.0])
    c = np.array([[10, 5, 10], [25, 10, 10], [40, 5, 10], [50, 15, 25]], float)
    u = 0.013
    d = O.OracleDem(box, c, r, vel=np.tile([u, 0.002, -0.001], (4, 1)), density=RHO, substeps=1)
    vol = 4.0 / 3.0 * math.pi * (r ** 3).sum()
    assert abs(d.bedload() - u * vol / (60 * 20)) < 1e-15
    v = np.zeros((4, 3))
    v[0, 0], v[2, 0], v[1, 0] = 0.01, -0.01, 0.004
    d = O.OracleDem(box, c, r, vel=v, fixed=[0, 0, 0, 1], density=RHO, substeps=1)
    assert abs(d.bedload() - 0.004 * 4.0 / 3.0 * math.pi * 27.0 / 1200) < 1e-16
    d2 = O.OracleDem(box, c, r, vel=2.5 * v, fixed=[0, 0, 0, 1], density=RHO, substeps=1)
    assert abs(d2.bedload() - 2.5 * d.bedload()) < 1e-16


def test_collision_across_the_periodic_seam():
    """Two spheres meeting across x = 0 collide as they would inside the box
    (minimum image), and their centres wrap back into [0, nx)."""
    u = 0.02
    box = (40, 40, 40)
    inside, _ = collide([[15.0, 20, 20], [25.2, 20, 20]], [5.0, 5.0], [[u, 0, 0], [-u, 0, 0]], box=box, steps=2000)
    d = O.OracleDem(box, [[34.9, 20, 20], [5.1, 20, 20]], [5.0, 5.0], vel=[[u, 0, 0], [-u, 0, 0]],
                    density=RHO, dt=0.05, substeps=1)
    for _ in range(2000):
        d.step()
    x, v, w = d.state()
    # the same collision: restitution e_dry, opposite velocities (the
    # wrapped separation rounds differently, which may move the contact's
    # first sub-step and the rebound speed by ~1e-4)
    assert abs(v[1, 0] / u - 0.97) < 5e-4 and abs(inside[1, 0] / u - 0.97) < 5e-4
    assert v[0, 0] == -v[1, 0] and not v[:, 1:].any()
    assert (x[:, 0] >= 0).all() and (x[:, 0] < 40).all()


def _slip_decay(d, slip, t1, h):
    """decay rate of the slip velocity over [0, t1]"""
    s0 = slip(d.state())
    for _ in range(int(round(t1 / h))):
        d.step()
    return -math.log(slip(d.state()) / s0) / t1


def test_tangential_lubrication_against_the_wall():
    """A sphere sliding along the wall inside the lubrication range (no
    contact, no gravity): the tangential force acts at the middle of the gap,
    so angular momentum about that point is conserved and the sphere ends
    rolling at v0 / (1 + I/(m l^2)), l = r + s/2; the slip v - l w decays
    at 6 pi mu (8 r/15) ln(s_c/s) (1/m + l^2/I) (Goldman, Cox and Brenner's
    coefficient for a sphere translating past a wall)."""
    r, s, mu, sc, v0, h = 5.0, 0.1, 0.1, 0.6, 0.01, 0.02
    ell = r + s / 2
    m = mass(r)
    inertia = 0.4 * m * r * r
    d = O.OracleDem((400, 50, 50), [[20, 25, r + s]], [r], vel=[[v0, 0, 0]], density=RHO, viscosity=mu,
                    lub_cut=sc, lub_min=1e-4, dt=h, substeps=1)
    slip = lambda st: st[1][0, 0] - ell * st[2][0, 1]      # noqa: E731
    k = _slip_decay(d, slip, 10.0, h)
    want = 6 * math.pi * mu * (8 * r / 15) * math.log(sc / s) * (1 / m + ell ** 2 / inertia)
    assert abs(k / want - 1) < 2e-3, (k, want)
    for _ in range(40000):
        d.step()
    x, v, w = d.state()
    assert abs(x[0, 2] - (r + s)) < 1e-12                 # the gap stays
    assert abs(v[0, 0] / v0 - 1 / (1 + inertia / (m * ell ** 2))) < 1e-4
    assert abs(ell * w[0, 1] / v[0, 0] - 1) < 1e-4


def test_tangential_lubrication_between_spheres():
    """Two equal spheres sliding past each other at a fixed gap: momentum is
    conserved and the slip decays at 6 pi mu (r/6) ln(s_c/s) (2/m + 2 l^2/I)
    (Jeffrey and Onishi's coefficient for equal spheres)."""
    r, s, mu, sc, v0, h = 5.0, 0.1, 0.1, 0.6, 0.01, 0.02
    ell = r + s / 2
    m = mass(r)
    inertia = 0.4 * m * r * r
    d = O.OracleDem((200, 200, 200), [[100, 100, 100], [100, 100, 100 + 2 * r + s]], [r, r],
                    vel=[[v0, 0, 0], [-v0, 0, 0]], density=RHO, viscosity=mu, lub_cut=sc, lub_min=1e-4,
                    dt=h, substeps=1)
    # slip of sphere 0's top point against sphere 1's bottom point
    slip = lambda st: (st[1][0, 0] + ell * st[2][0, 1]) - (st[1][1, 0] - ell * st[2][1, 1])  # noqa: E731
    k = _slip_decay(d, slip, 10.0, h)
    want = 6 * math.pi * mu * (r / 6) * math.log(sc / s) * (2 / m + 2 * ell ** 2 / inertia)
    assert abs(k / want - 1) < 2e-3, (k, want)
    x, v, w = d.state()
    assert abs(v[:, 0].sum()) < 1e-17 and abs(v[:, 2].sum()) < 1e-17
