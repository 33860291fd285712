"""Pins of the oracle's momentum-exchange force and torque on spheres.

Section 2.2 couples fluid and particles by momentum exchange (citing Aidun
et al. 1998 and Wen et al. 2014; the oracle takes Wen's Galilean-invariant
form at the link midpoints).  The checks below do not retype that formula:

* fluid at rest around any solid set (overlapping spheres, off-centre):
  force and torque vanish -- each solid cell's links cancel in pairs;
* a sphere translating through fluid at rest: the force is linear in U and
  opposes it, -6 sum_links w_j c_j (c_j . U) with the links enumerated here
  independently; no transverse force and no torque for a sphere centred on
  a cell centre (cubic symmetry);
* a sphere rotating in fluid at rest: no force, torque against the spin;
* a sphere at rest cut by a free surface, fluid at rest: the force is the
  rest pressure -2 sum w_j c_j over the links from liquid and interface
  cells (gas cells exchange nothing), links enumerated here;
* momentum balance over one step of an all-liquid box without body force:
  the fluid's momentum changes by minus the total force on resting spheres
  (exactly, up to rounding), and for moving spheres by minus the force plus
  the Galilean correction sum_links 6 w_j u_w (c_j . u_w), summed here over
  an independent link enumeration.
"""
import numpy as np
import pytest

from oracle import oracle as O

pytestmark = pytest.mark.filterwarnings("ignore")

C, W = O.velocities()


def box(shape, vel=None):
    nx, ny, nz = shape
    fill = np.ones((nz, ny, nx))
    rho = np.ones((nz, ny, nx))
    return O.OracleLattice(shape, 1.6, fill=fill, rho=rho, vel=vel)


def links(o, centre, radius, types=(O.LIQUID,)):
    """(cell z, y, x, direction j, sphere q, midpoint offset r) of every link
    from a cell of the given types into a sphere, by brute force over cells
    and directions."""
    nx, ny, nz = o.shape
    t = o.read(O.F_TYPE)
    own = o.read(O.F_OWNER)
    out = []
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                if t[z, y, x] not in types:
                    continue
                for j in range(27):
                    if j == 13:
                        continue
                    sx, sy, sz = x - C[j][0], y - C[j][1], z - C[j][2]
                    if sz < 0 or sz >= nz:
                        continue
                    sx %= nx
                    sy %= ny
                    if t[sz, sy, sx] != O.SOLID:
                        continue
                    q = own[sz, sy, sx]
                    r = np.array([x + 0.5 - 0.5 * C[j][0], y + 0.5 - 0.5 * C[j][1],
                                  z + 0.5 - 0.5 * C[j][2]]) - centre[q]
                    r[0] -= nx * np.round(r[0] / nx)
                    r[1] -= ny * np.round(r[1] / ny)
                    out.append((z, y, x, j, q, r))
    return out


def momentum(o):
    f = o.read(O.F_PDF)
    t = o.read(O.F_TYPE)
    liq = t == O.LIQUID
    return np.array([(C[:, a][:, None] * f[:, liq]).sum() for a in range(3)])


def test_rest_gives_no_force_for_any_solid_set():
    o = box((20, 18, 22))
    centre = np.array([[7.3, 8.1, 9.6], [10.2, 9.4, 11.9], [14.7, 5.2, 10.4]])
    o.set_particles(centre, [3.4, 2.9, 2.2])
    ft = o.particle_forces()
    assert ft.shape == (3, 6)
    # a single link carries about 2 w ~ 0.07; the sums cancel to rounding.
    # The cancellation holds per connected solid set: the first two spheres
    # overlap (their cells where they touch have no fluid links), so only
    # their total force and their total torque about a common point vanish.
    assert np.abs(ft[2]).max() < 1e-14, ft[2]
    pair = ft[:2]
    assert np.abs(pair[:, :3]).max() > 0.1
    assert np.abs(pair[:, :3].sum(0)).max() < 1e-14
    torque = pair[:, 3:].sum(0) + np.cross(centre[:2], pair[:, :3]).sum(0)
    assert np.abs(torque).max() < 1e-13, torque


def test_translating_sphere_drag():
    o = box((16, 16, 16))
    centre = np.array([[8.5, 8.5, 8.5]])
    U = np.array([2e-3, 0.0, 0.0])
    o.set_particles(centre, [3.3], vel=U[None, :])
    ft = o.particle_forces()[0]
    lk = links(o, centre, None)
    assert len(lk) > 100
    M = np.zeros((3, 3))
    for (_, _, _, j, _, _) in lk:
        M += W[j] * np.outer(C[j], C[j])
    expect = -6.0 * M @ U
    # the rest-state parts (about 2 w per link) cancel to rounding, 1e-14
    assert np.allclose(ft[:3], expect, rtol=1e-12, atol=1e-14), (ft[:3], expect)
    assert ft[0] < -0.1
    assert abs(ft[1]) < 1e-14 and abs(ft[2]) < 1e-14
    assert np.abs(ft[3:]).max() < 1e-13


def test_rotating_sphere_torque_opposes_spin():
    o = box((16, 16, 16))
    centre = np.array([[8.5, 8.5, 8.5]])
    Om = np.array([0.0, 0.0, 1e-3])
    o.set_particles(centre, [3.3], angvel=Om[None, :])
    ft = o.particle_forces()[0]
    assert np.abs(ft[:3]).max() < 1e-14, ft
    assert abs(ft[3]) < 1e-13 and abs(ft[4]) < 1e-13
    assert ft[5] < -1e-3


def test_partially_submerged_sphere_at_rest():
    shape = (18, 16, 20)
    nx, ny, nz = shape
    z = np.arange(nz)[:, None, None] + np.zeros((nz, ny, nx))
    fill = np.clip(10.4 - z, 0.0, 1.0)  # liquid below z = 10.4, one interface layer
    o = O.OracleLattice(shape, 1.6, fill=fill, rho=np.ones((nz, ny, nx)))
    centre = np.array([[8.7, 7.9, 10.1]])
    o.set_particles(centre, [3.6])
    t = o.read(O.F_TYPE)
    assert (t == O.INTERFACE).sum() > 50
    ft = o.particle_forces()[0]
    lk = links(o, centre, None, types=(O.LIQUID, O.INTERFACE))
    assert any(t[zz, yy, xx] == O.INTERFACE for (zz, yy, xx, _, _, _) in lk)
    F = np.zeros(3)
    T = np.zeros(3)
    for (_, _, _, j, _, r) in lk:
        Fl = -2.0 * W[j] * C[j]
        F += Fl
        T += np.cross(r, Fl)
    assert np.allclose(ft[:3], F, rtol=0, atol=1e-13), (ft[:3], F)
    assert np.allclose(ft[3:], T, rtol=0, atol=1e-12), (ft[3:], T)
    # the submerged part is pushed up by the liquid below
    assert ft[2] > 0.1


def blob_velocity(shape, centre, radius, amp):
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5, np.arange(nx) + 0.5, indexing="ij")
    d2 = (x - centre[0]) ** 2 + (y - centre[1]) ** 2 + (z - centre[2]) ** 2
    s = np.where(d2 < radius ** 2, (1.0 - d2 / radius ** 2) ** 2, 0.0)
    return np.stack([amp[0] * s, amp[1] * s, amp[2] * s])


@pytest.mark.parametrize("moving", [False, True])
def test_momentum_balance_over_one_step(moving):
    shape = (24, 22, 26)
    vel = blob_velocity(shape, (12.0, 11.0, 13.0), 7.0, (0.02, -0.013, 0.008))
    o = box(shape, vel=vel)
    centre = np.array([[11.2, 10.7, 12.6], [14.1, 12.3, 14.9]])
    radius = [2.6, 2.1]
    sv = np.array([[1e-3, -2e-3, 5e-4], [-8e-4, 1e-3, 0.0]]) if moving else None
    sw = np.array([[2e-4, -1e-4, 3e-4], [0.0, 4e-4, -2e-4]]) if moving else None
    o.set_particles(centre, radius, vel=sv, angvel=sw)
    ft = o.particle_forces()
    p0 = momentum(o)
    corr = np.zeros(3)
    if moving:
        for (_, _, _, j, q, r) in links(o, centre, radius):
            uw = sv[q] + np.cross(sw[q], r)
            corr += 6.0 * W[j] * uw * (C[j] @ uw)
    o.step(1)
    p1 = momentum(o)
    # the fluid loses what the spheres gain by plain momentum exchange; the
    # Galilean-invariant form adds the correction to the spheres' side
    lhs = ft[:, :3].sum(0)
    rhs = -(p1 - p0) + corr
    # rounding: the momentum sums run over ~1e4 cells, and the z walls (fluid
    # at rest there) exchange +-1/3 per wall cell, which cancels between the
    # bottom and top rows only to ~1e-13
    assert np.allclose(lhs, rhs, rtol=0, atol=1e-12), (lhs, rhs)
    assert np.abs(lhs).max() > 1e-5
