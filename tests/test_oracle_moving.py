"""Pins of the oracle's moving spheres (remapping the lattice when spheres
move; Section 2.2 resolves moving particles on the lattice, the remapping
rules are readings).

* the total mass (cells plus pool) is exact over moves and steps, with a
  free surface;
* a sphere moved by whole cells through liquid at rest: the solid cells
  are the old ones shifted, and every uncovered cell has density 1 and the
  sphere's rigid-body velocity at its centre;
* a sphere lifted out of a film: cells uncovered above the surface are gas,
  no liquid cell ever touches a gas cell, the film keeps its mass;
* a sphere dropped from the gas into a film: the cells uncovered in one
  round next to cells typed gas in the same round are interface cells, no
  liquid cell touches a gas cell, and the mass stays exact;
* moving back to the start gives back the original solid cells.
"""
import numpy as np

from oracle import oracle as O


def liquid_box(shape, omega=1.4):
    nx, ny, nz = shape
    return O.OracleLattice(shape, omega, fill=np.ones((nz, ny, nx)))


def no_liquid_next_to_gas(t):
    liq, gas = t == O.LIQUID, t == O.GAS
    nz = t.shape[0]
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                sh = np.roll(np.roll(gas, dy, 1), dx, 2)
                if dz == 1:
                    sh = np.concatenate([np.zeros_like(sh[:1]), sh[:-1]], 0)
                elif dz == -1:
                    sh = np.concatenate([sh[1:], np.zeros_like(sh[:1])], 0)
                if np.any(liq & sh):
                    return False
    return True


def test_integer_shift_through_liquid_at_rest():
    shape = (20, 16, 18)
    o = liquid_box(shape)
    c0 = np.array([[8.3, 7.6, 8.9]])
    U = np.array([[2e-3, -1e-3, 5e-4]])
    W = np.array([[1e-4, 2e-4, -3e-4]])
    o.set_particles(c0, [3.6], vel=U, angvel=W)
    s0 = o.read(O.F_TYPE) == O.SOLID
    shift = np.array([2, -1, 1])
    o.move_particles(c0 + shift, vel=U, angvel=W)
    t = o.read(O.F_TYPE)
    s1 = t == O.SOLID
    expect = np.roll(np.roll(np.roll(s0, shift[2], 0), shift[1], 1), shift[0], 2)
    assert np.array_equal(s1, expect)
    uncovered = s0 & ~s1
    assert uncovered.sum() > 10
    assert np.all(t[uncovered] == O.LIQUID)
    rho = o.read(O.F_RHO)[uncovered]
    assert np.allclose(rho, 1.0, rtol=0, atol=1e-14)
    nz, ny, nx = t.shape
    z, y, x = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5, np.arange(nx) + 0.5, indexing="ij")
    r = np.stack([x - c0[0, 0] - shift[0], y - c0[0, 1] - shift[1], z - c0[0, 2] - shift[2]])
    uw = U[0][:, None] + np.cross(W[0], r[:, uncovered].T).T
    assert np.allclose(o.read(O.F_VEL)[:, uncovered], uw, rtol=0, atol=1e-15)


def test_mass_exact_over_moves_and_steps():
    shape = (24, 12, 20)
    nx, ny, nz = shape
    z = np.arange(nz)[:, None, None] + np.zeros((nz, ny, nx))
    fill = np.clip(12.3 - z, 0.0, 1.0)
    o = O.OracleLattice(shape, 1.5, accel=(1e-5, 0.0, -1e-5), fill=fill)
    c = np.array([[6.0, 6.0, 5.0], [15.5, 4.2, 11.0]])
    o.set_particles(c, [2.6, 2.2])
    M0 = o.total_mass()
    rng = np.random.default_rng(4)
    for k in range(12):
        c = c + rng.uniform(-0.7, 0.7, size=c.shape)
        c[:, 2] = np.clip(c[:, 2], 3.5, 15.0)
        o.move_particles(c, vel=rng.normal(0, 1e-3, size=c.shape))
        o.step(3)
        assert abs(o.total_mass() - M0) <= 1e-12 * M0
        assert no_liquid_next_to_gas(o.read(O.F_TYPE))


def test_sphere_lifted_out_of_a_film():
    shape = (16, 16, 24)
    nx, ny, nz = shape
    z = np.arange(nz)[:, None, None] + np.zeros((nz, ny, nx))
    fill = np.clip(10.5 - z, 0.0, 1.0)
    o = O.OracleLattice(shape, 1.5, fill=fill)
    c0 = np.array([[8.0, 8.0, 10.0]])
    o.set_particles(c0, [3.4])
    s0 = o.read(O.F_TYPE) == O.SOLID
    M0 = o.total_mass()
    o.move_particles(c0 + np.array([0.0, 0.0, 8.0]))
    t = o.read(O.F_TYPE)
    uncovered = s0 & (t != O.SOLID)
    zc = np.broadcast_to(np.arange(nz)[:, None, None], t.shape)
    assert np.all(t[uncovered & (zc >= 12)] == O.GAS)
    assert np.any(t[uncovered] == O.LIQUID)
    assert no_liquid_next_to_gas(t)
    assert abs(o.total_mass() - M0) <= 1e-12 * M0


def test_sphere_dropped_from_the_gas_into_a_film():
    """A sphere above the surface dropped into the liquid: the cells it
    uncovers just above the surface are typed in one round, some liquid
    (liquid neighbours below) next to others gas (gas neighbours above);
    the liquid ones become interface cells, so that no liquid cell
    borders gas, and the total mass stays exact over the following
    steps."""
    shape = (22, 16, 28)
    nx, ny, nz = shape
    z = np.arange(nz)[:, None, None] + np.zeros((nz, ny, nx))
    fill = np.clip(17.2 - z, 0.0, 1.0)
    o = O.OracleLattice(shape, 1.5, accel=(1e-5, 0.0, -1e-5), fill=fill, conv_eps=1e-3)
    c = np.array([[6.3, 8.2, 20.0], [15.5, 6.0, 15.0]])
    o.set_particles(c, [2.4, 2.1])
    M0 = o.total_mass()
    o.move_particles(c + np.array([[0.0, 0.0, -13.0], [0.0, 0.3, -7.5]]), vel=np.full((2, 3), 1e-3))
    assert no_liquid_next_to_gas(o.read(O.F_TYPE))
    for _ in range(4):
        o.step(2)
        assert abs(o.total_mass() - M0) <= 1e-12 * M0
        assert no_liquid_next_to_gas(o.read(O.F_TYPE))


def test_round_trip_restores_the_solid_cells():
    shape = (18, 14, 16)
    o = liquid_box(shape)
    c0 = np.array([[5.2, 6.9, 7.7], [12.6, 3.1, 8.4]])
    o.set_particles(c0, [2.9, 2.4])
    s0 = o.read(O.F_TYPE) == O.SOLID
    own0 = o.read(O.F_OWNER)
    o.move_particles(c0 + np.array([[1.7, -0.4, 0.9], [-2.2, 3.3, -1.1]]))
    assert not np.array_equal(o.read(O.F_TYPE) == O.SOLID, s0)
    o.move_particles(c0)
    assert np.array_equal(o.read(O.F_TYPE) == O.SOLID, s0)
    assert np.array_equal(o.read(O.F_OWNER), own0)
