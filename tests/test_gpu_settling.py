"""A sphere settling through liquid, run by the coupled step (fluid step,
momentum-exchange force, particle sub-steps, remap) on the GPU.

Physics, not parity: the sphere (density 1.5) starts at rest in liquid at
rest with the hydrostatic density of the body force, accelerates and reaches
a terminal velocity.  There the hydrodynamic force carries its weight
(buoyancy plus drag), and the velocity lies below Stokes' 2(rho_p - 1) g r^2
/ (9 nu) by the hindrance of the periodic box and the walls, but within a
factor two of it.  A wrong sign of the force or of the wall velocity in the
bounce-back would make it accelerate without bound.
"""
import math

import numpy as np
import pytest

from paper_2301_10674_amd import inputs as I

pytestmark = pytest.mark.gpu


def test_sphere_reaches_terminal_velocity():
    from paper_2301_10674_amd import fsl
    from paper_2301_10674_amd.couple import Coupled

    nx, ny, nz = 40, 40, 56
    g, r, rho_p, omega = 4e-5, 4.0, 1.5, 1.2
    nu = (1 / omega - 0.5) / 3
    z = np.arange(nz)[:, None, None] + 0.5 + np.zeros((nz, ny, nx))
    rho = np.exp(3 * g * (nz - z))
    w = I.Workload(name="settle", shape=(nx, ny, nz), omega=omega, accel=(0.0, 0.0, -g), sigma=0.0,
                   fill=np.ones((nz, ny, nx)), rho=rho, vel=np.zeros((3, nz, ny, nx)),
                   centre=np.array([[20.3, 19.8, 38.0]]), radius=np.array([r]),
                   sphere_vel=np.zeros((1, 3)), sphere_angvel=np.zeros((1, 3)))
    lat = fsl.lattice_from_workload(w, "fp64")
    dem = fsl.Dem(w.shape, w.centre, w.radius, None, None, None, density=rho_p, viscosity=nu,
                  lub_cut=0.6, accel=(0.0, 0.0, -g), substeps=5, skin=1.0)
    run = Coupled(lat, dem)
    vz, fz = [], []
    for _ in range(60):
        run.step(10)
        vz.append(dem.state()[1][0, 2])
        fz.append(lat.particle_forces()[0, 2])
    vz, fz = np.array(vz), np.array(fz)
    m = rho_p * 4 / 3 * math.pi * r ** 3
    u_stokes = 2 * (rho_p - 1) * g * r ** 2 / (9 * nu)
    tail = slice(40, 60)
    u = -vz[tail].mean()
    print("terminal velocity %.3e (Stokes %.3e), hydrodynamic force %.4f against weight %.4f" % (
        u, u_stokes, fz[tail].mean(), m * g))
    assert vz[tail].max() < 0                                  # falling
    assert np.abs(np.diff(vz[tail])).max() < 0.02 * u          # steady
    assert abs(fz[tail].mean() / (m * g) - 1) < 0.02           # force carries the weight
    assert 0.5 < u / u_stokes < 1.0
    assert dem.state()[0][0, 2] < 38.0 - 0.5 * u * 400         # it moved
    lat.destroy()
    dem.destroy()
