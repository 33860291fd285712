"""GPU parity of the momentum-exchange force and torque (fsl_particle_forces)
against the oracle's, through the C-ABI.

* FP64: spheres that move, rotate and wrap across the periodic x/y
  boundaries in a small liquid box, and the flume recipe (128 x 40 x 192
  crop, a free surface over three layers of spheres), after several steps;
  per sphere, agreement to 1e-11 of the largest link-sum magnitude (the
  sums cancel terms of about 2 w per link).
* FP32 and FP16 storage against the FP64 oracle on the flume crop: the
  per-sphere forces differ by the storage rounding of the PDFs summed over
  a sphere's links.
* Repeated evaluation and a repeated run give bit-identical results (fixed
  summation order); no spheres: nothing to compute; argument errors.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2301_10674_amd import inputs as I

pytestmark = pytest.mark.gpu


def F():
    from paper_2301_10674_amd import fsl
    return fsl


def oracle_from(w, **kw):
    L = O.OracleLattice(w.shape, w.omega, accel=w.accel, sigma=w.sigma, rho_gas=w.rho_gas,
                        conv_eps=w.conv_eps, fill=w.fill, rho=w.rho, vel=w.vel, **kw)
    L.set_particles(w.centre, w.radius, w.sphere_vel, w.sphere_angvel)
    return L


def spinning_box():
    nx, ny, nz = 14, 12, 14
    rng = np.random.default_rng(11)
    return I.Workload(name="box", shape=(nx, ny, nz), omega=1.7, accel=(1e-5, 2e-6, -3e-6),
                      sigma=0.0, fill=np.ones((nz, ny, nx)),
                      rho=1 + 0.01 * rng.standard_normal((nz, ny, nx)),
                      vel=0.01 * rng.standard_normal((3, nz, ny, nx)),
                      centre=np.array([[3.0, 4.0, 5.0], [9.5, 7.2, 7.1], [13.7, 0.3, 3.0]]),
                      radius=np.array([2.5, 3.0, 2.2]),
                      sphere_vel=np.array([[1e-3, 0, -1e-3], [0, 2e-3, 0], [5e-4, 5e-4, 5e-4]]),
                      sphere_angvel=np.array([[0, 0, 1e-3], [1e-3, 0, 0], [2e-4, -3e-4, 1e-4]]))


def compare(gft, oft, rel):
    scale = np.abs(oft).max()
    err = np.abs(gft - oft).max()
    print("max |F, T| %.3e, max difference %.3e" % (scale, err))
    assert err <= rel * max(scale, 1.0), (err, scale)


@pytest.mark.parametrize("steps", [0, 7])
def test_spinning_spheres_fp64(steps):
    w = spinning_box()
    g = F().lattice_from_workload(w, "fp64")
    o = oracle_from(w)
    g.step(steps)
    o.step(steps)
    gft = g.particle_forces()
    g.destroy()
    oft = o.particle_forces()
    assert gft.shape == (3, 6)
    compare(gft, oft, 1e-11)


def test_flume_crop_fp64():
    w = I.flume_crop(nx=128, seed=3)
    O.set_threads(0)
    g = F().lattice_from_workload(w, "fp64")
    o = oracle_from(w)
    g.step(5)
    o.step(5)
    gft = g.particle_forces()
    g.destroy()
    oft = o.particle_forces()
    assert gft.shape == (len(w.radius), 6)
    assert np.abs(oft[:, :3]).max() > 1e-3
    compare(gft, oft, 1e-11)


@pytest.mark.parametrize("prec,rel", [("fp32", 1e-5), ("fp16", 3e-3)])
def test_flume_crop_reduced_storage(prec, rel):
    w = I.flume_crop(nx=128, seed=3)
    O.set_threads(0)
    g = F().lattice_from_workload(w, prec)
    o = oracle_from(w)
    g.step(5)
    o.step(5)
    gft = g.particle_forces()
    g.destroy()
    compare(gft, o.particle_forces(), rel)


def test_deterministic():
    w = spinning_box()
    runs = []
    for _ in range(2):
        g = F().lattice_from_workload(w, "fp32")
        g.step(5)
        a = g.particle_forces()
        b = g.particle_forces()
        g.destroy()
        assert np.array_equal(a, b)
        runs.append(a)
    assert np.array_equal(runs[0], runs[1])


def test_no_spheres_and_errors():
    f = F()
    nx, ny, nz = 8, 6, 8
    w = I.Workload(name="plain", shape=(nx, ny, nz), omega=1.5, accel=(0, 0, 0), sigma=0.0,
                   fill=np.ones((nz, ny, nx)), rho=np.ones((nz, ny, nx)), vel=None,
                   centre=np.zeros((0, 3)), radius=np.zeros(0), sphere_vel=np.zeros((0, 3)),
                   sphere_angvel=np.zeros((0, 3)))
    g = f.lattice_from_workload(w, "fp64")
    assert g.particle_forces().shape == (0, 6)
    assert f.lib().fsl_particle_forces(None, None, 0) == f.FSL_ERR_STATE
    g.destroy()
    g = f.lattice_from_workload(spinning_box(), "fp64")
    assert f.lib().fsl_particle_forces(g.h, None, 0) == f.FSL_ERR_ARG
    g.destroy()
