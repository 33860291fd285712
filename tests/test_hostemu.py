"""The library's kernels built as host code (tests/hostemu: a CPU stand-in
for the HIP runtime, kernels unchanged but for launch syntax) run against
the FP64 oracle on the CPU, under UBSan with array-bounds checks.

This checks the kernel sources on their own, apart from the GPU compiler:
the GPU parity tests compare what the GPU compiler made of them.  The cases
are those where the GPU build has gone wrong before -- lattices three and
five cells high (every cell neighbours every cell of the next row, filled
cells share their excess with a whole row) with and without the Galilean
correction, and a film whose crests touch the top wall -- so that a
difference between the GPU and the oracle there can be placed: in the
source if this test fails too, in the compiled code if it does not.  The
moving spheres are checked here too (remaps, refilled link lists, spheres
jumping through the surface, random moves), since their kernels are long
chains of list passes that are easiest to check bounds-checked.
"""
import dataclasses
import os
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2301_10674_amd import fsl as F
from paper_2301_10674_amd import inputs as I

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "hostemu"))
import emu  # noqa: E402


def tiny(shape, h):
    nx, ny, nz = shape
    xc = np.arange(nx) + 0.5
    hh = h + 0.7 * np.sin(2 * np.pi * xc / nx)
    fill = I.height_fill(shape, np.broadcast_to(hh[None, :], (ny, nx)))
    rng = np.random.default_rng(5)
    return I.Workload(name="tiny", shape=shape, omega=1.3, accel=(1e-4, 0, -1e-4), sigma=1e-3,
                      fill=fill, rho=np.ones((nz, ny, nx)), vel=0.01 * rng.standard_normal((3, nz, ny, nx)),
                      centre=np.zeros((0, 3)), radius=np.zeros(0), sphere_vel=np.zeros((0, 3)),
                      sphere_angvel=np.zeros((0, 3)))


def lid():
    w = I.film_with_surface_spheres(nz=22, sigma=1e-3)
    return dataclasses.replace(w, centre=w.centre[:18], radius=w.radius[:18], sphere_vel=w.sphere_vel[:18],
                               sphere_angvel=w.sphere_angvel[:18])


def compare(g, o, label):
    t = o.read(O.F_TYPE)
    assert np.array_equal(g.read(F.FIELD_TYPE), t), label
    fl = (t == O.LIQUID) | (t == O.INTERFACE)
    for gf, of in ((F.FIELD_MASS, O.F_MASS), (F.FIELD_FILL, O.F_FILL)):
        assert np.abs(g.read(gf)[fl] - o.read(of)[fl]).max() <= 1e-12, (label, gf)
    assert np.abs(g.read(F.FIELD_PDF)[:, fl] - o.read(O.F_PDF)[:, fl]).max() <= 1e-12, label


@pytest.mark.parametrize("galilean", [False, True])
@pytest.mark.parametrize("shape,h", [((3, 3, 3), 1.6), ((6, 3, 3), 1.6), ((3, 3, 5), 2.6)])
def test_tiny_lattices_on_the_cpu(shape, h, galilean):
    w = tiny(shape, h)
    kw = dict(galilean=True) if galilean else {}
    g = emu.EmuLattice(w, "fp64", **kw)
    o = O.OracleLattice(w.shape, w.omega, accel=w.accel, sigma=w.sigma, fill=w.fill, rho=w.rho, vel=w.vel, **kw)
    for k in range(4):
        g.step(5)
        o.step(5)
        compare(g, o, "%s after %d steps" % (shape, 5 * (k + 1)))
    assert np.array_equal(g.counters()[:7], o.counters()[:7])
    g.destroy()


def test_surface_at_the_top_wall_on_the_cpu():
    w = lid()
    g = emu.EmuLattice(w, "fp64")
    o = O.OracleLattice(w.shape, w.omega, accel=w.accel, sigma=w.sigma, fill=w.fill, rho=w.rho, vel=w.vel)
    o.set_particles(w.centre, w.radius, w.sphere_vel, w.sphere_angvel)
    for k in range(3):
        g.step(2)
        o.step(2)
        compare(g, o, "lid after %d steps" % (2 * (k + 1)))
    assert o.counters()[2] > 0                 # cells filled next to the wall
    g.destroy()


def test_refilled_link_lists_on_the_cpu():
    """Momentum-exchange lists refilled only for the spheres a remap
    touched (a sphere crossing x = 0, one leaving the sphere it sat inside,
    so that its list outgrows its slot) against lists built from scratch
    after the same moves (bit-identical) and against the oracle's forces."""
    nx, ny, nz = 20, 16, 16
    z = np.arange(nz)[:, None, None] + np.zeros((nz, ny, nx))
    c0 = np.array([[1.2, 6.0, 5.0], [12.0, 6.0, 6.0], [12.0, 6.0, 6.0]])
    w = I.Workload(name="moving", shape=(nx, ny, nz), omega=1.6, accel=(2e-5, 0.0, -1e-5), sigma=0.0,
                   fill=np.clip(11.4 - z, 0.0, 1.0), rho=np.ones((nz, ny, nx)), vel=np.zeros((3, nz, ny, nx)),
                   centre=c0, radius=np.array([2.3, 1.6, 3.0]), sphere_vel=np.full((3, 3), 1e-3),
                   sphere_angvel=np.zeros((3, 3)))
    moves = [np.array([[-0.45, 0.1, 0.0], [0.0, 0.0, 0.0], [0.2, -0.3, 0.1]]),
             np.array([[-0.45, -0.2, 0.05], [-5.5, 0.0, 2.0], [0.01, 0.02, -0.01]]),
             np.array([[-0.45, 0.3, 0.0], [0.3, 0.2, 0.0], [-0.4, 0.1, 0.0]])]
    vel = np.full((3, 3), 1e-3)
    a = emu.EmuLattice(w, "fp64")
    o = O.OracleLattice(w.shape, w.omega, accel=w.accel, fill=w.fill, rho=w.rho, vel=w.vel, conv_eps=w.conv_eps)
    o.set_particles(w.centre, w.radius, w.sphere_vel, w.sphere_angvel)
    a.step(2)
    o.step(2)
    a.particle_forces(3)
    c = c0.copy()
    got = []
    for d in moves:
        c = c + d
        a.move_particles(c, vel)
        o.move_particles(c, vel)
        a.step(1)
        o.step(1)
        fa, fo = a.particle_forces(3), o.particle_forces()
        assert np.abs(fa - fo).max() <= 1e-11 * max(np.abs(fo).max(), 1.0)
        got.append(fa)
    a.destroy()
    b = emu.EmuLattice(w, "fp64")
    b.step(2)
    c = c0.copy()
    for d in moves:
        c = c + d
        b.move_particles(c, vel)
        b.step(1)
    assert np.array_equal(b.particle_forces(3), got[-1])
    b.destroy()


def test_spheres_jumping_through_the_surface_on_the_cpu():
    """Spheres moved several cells up into the gas and back down into the
    liquid (the uncovering rounds type cells liquid next to cells typed
    gas in the same round, which the closure makes interface cells),
    against the oracle after each move and after steps: types, masses, fill
    levels and PDFs to 1e-12, the total mass exact."""
    nx, ny, nz = 22, 16, 28
    z = np.arange(nz)[:, None, None] + np.zeros((nz, ny, nx))
    c = np.array([[6.0, 8.0, 5.5], [15.0, 6.0, 6.0]])
    w = I.Workload(name="jumps", shape=(nx, ny, nz), omega=1.5, accel=(1e-5, 0.0, -1e-5), sigma=0.0,
                   fill=np.clip(17.2 - z, 0.0, 1.0), rho=np.ones((nz, ny, nx)), vel=np.zeros((3, nz, ny, nx)),
                   centre=c, radius=np.array([2.4, 2.1]), sphere_vel=np.zeros((2, 3)),
                   sphere_angvel=np.zeros((2, 3)))
    g = emu.EmuLattice(w, "fp64")
    o = O.OracleLattice(w.shape, w.omega, accel=w.accel, fill=w.fill, rho=w.rho, vel=w.vel, conv_eps=w.conv_eps)
    o.set_particles(w.centre, w.radius, w.sphere_vel, w.sphere_angvel)
    M0 = o.total_mass()
    jumps = [[[0.3, 0.0, 6.5], [0.0, -0.4, 0.0]], [[0.0, 0.2, 8.0], [0.5, 0.0, 9.0]],
             [[0.0, 0.0, -13.0], [0.0, 0.3, -7.5]]]
    for k, dj in enumerate(jumps):
        c = c + np.array(dj)
        v = np.full(c.shape, 1e-3)
        g.move_particles(c, v)
        o.move_particles(c, v)
        compare(g, o, "jump %d" % k)
        g.step(3)
        o.step(3)
        compare(g, o, "jump %d + 3 steps" % k)
        assert abs(g.total_mass() - M0) <= 1e-12 * M0
    g.destroy()


def test_random_moves_through_the_surface_on_the_cpu():
    """Three spheres in a film, moved at random by a fraction of a cell or
    by several cells (through the surface, into the gas and the liquid),
    with steps between: against the oracle after every move and step,
    the total mass exact."""
    rng = np.random.default_rng(101)
    nx, ny, nz = 18, 14, 22
    z = np.arange(nz)[:, None, None] + np.zeros((nz, ny, nx))
    n = 3
    c = np.stack([(2.0 + np.arange(n) * nx / n) % nx, rng.uniform(0, ny, n), rng.uniform(4, nz - 5, n)], 1)
    r = rng.uniform(1.6, 2.6, n)
    w = I.Workload(name="random", shape=(nx, ny, nz), omega=1.5, accel=(1e-5, 0.0, -1e-5), sigma=0.0,
                   fill=np.clip(11.6 - z, 0.0, 1.0), rho=np.ones((nz, ny, nx)), vel=np.zeros((3, nz, ny, nx)),
                   centre=c, radius=r, sphere_vel=np.zeros((n, 3)), sphere_angvel=np.zeros((n, 3)))
    g = emu.EmuLattice(w, "fp64")
    o = O.OracleLattice(w.shape, w.omega, accel=w.accel, fill=w.fill, rho=w.rho, vel=w.vel, conv_eps=w.conv_eps)
    o.set_particles(c, r, w.sphere_vel, w.sphere_angvel)
    M0 = o.total_mass()
    for k in range(5):
        far = k % 2 == 0
        c = c + (rng.uniform(-6, 6, size=(n, 3)) if far else rng.uniform(-0.6, 0.6, size=(n, 3)))
        c[:, 2] = np.clip(c[:, 2], 3.0, nz - 4.0)
        v = rng.normal(0, 1e-3, size=(n, 3))
        g.move_particles(c, v)
        o.move_particles(c, v)
        compare(g, o, "move %d" % k)
        g.step(2)
        o.step(2)
        compare(g, o, "move %d + 2 steps" % k)
        assert abs(g.total_mass() - M0) <= 1e-12 * M0
    g.destroy()


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("fp16", 2e-3)])
def test_storage_forms_on_the_cpu(prec, tol):
    """The FP32 and FP16 forms (whose dense pass reads and writes its rows
    through buffer descriptors, bounds-checked here) against the oracle
    storing the same precision: to a few units of the storage rounding."""
    w = lid()
    g = emu.EmuLattice(w, prec)
    o = O.OracleLattice(w.shape, w.omega, accel=w.accel, sigma=w.sigma, fill=w.fill, rho=w.rho, vel=w.vel,
                        store=prec)
    o.set_particles(w.centre, w.radius, w.sphere_vel, w.sphere_angvel)
    g.step(4)
    o.step(4)
    t = o.read(O.F_TYPE)
    assert np.array_equal(g.read(F.FIELD_TYPE), t)
    fl = (t == O.LIQUID) | (t == O.INTERFACE)
    d = np.abs(g.read(F.FIELD_PDF)[:, fl] - o.read(O.F_PDF)[:, fl]).max()
    assert d <= tol, d
    g.destroy()
