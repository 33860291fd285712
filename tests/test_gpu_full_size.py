"""Parity at the full benchmark sizes, in the configuration the benchmark runs.

* The flume 1536 x 40 x 192 (1848 spheres) and the large flume
  3072 x 80 x 256 (9210 spheres): the GPU in FP64 against the FP64 oracle
  after a few steps, over every cell that is fluid in both (the oracle runs
  its per-cell phases on all host threads), and the momentum-exchange force
  and torque on every sphere; the particle step on the large flume's bed
  (to 1e-12 of the oracle's all-pairs evaluation).
* The FP32 and FP16 forms on the 1536 x 40 x 192 flume over 200 steps:
  properties that hold at any size -- total mass conserved to 1e-12, no
  liquid cell next to a gas cell, fill levels of interface cells finite,
  every interface normal a unit vector or zero.
"""
import functools

import numpy as np
import pytest

from oracle import oracle as O
from paper_2301_10674_amd import inputs as I

pytestmark = pytest.mark.gpu


def F():
    from paper_2301_10674_amd import fsl
    return fsl


def compare_fp64(w, steps):
    f = F()
    O.set_threads(0)
    o = O.OracleLattice(w.shape, w.omega, accel=w.accel, sigma=w.sigma, rho_gas=w.rho_gas,
                        conv_eps=w.conv_eps, fill=w.fill, rho=w.rho, vel=w.vel)
    o.set_particles(w.centre, w.radius, w.sphere_vel, w.sphere_angvel)
    o.step(steps)
    g = f.lattice_from_workload(w, "fp64")
    g.step(steps)
    gf = g.read_fields([f.FIELD_TYPE, f.FIELD_VEL, f.FIELD_MASS])
    gft = g.particle_forces()
    g.destroy()
    to = o.read(O.F_TYPE)
    assert np.array_equal(gf[f.FIELD_TYPE], to)
    fluid = (to == O.LIQUID) | (to == O.INTERFACE)
    dv = np.abs(gf[f.FIELD_VEL][:, fluid] - o.read(O.F_VEL)[:, fluid]).max()
    dm = np.abs(gf[f.FIELD_MASS][fluid] - o.read(O.F_MASS)[fluid]).max()
    # momentum-exchange force and torque on every sphere
    oft = o.particle_forces()
    df = np.abs(gft - oft).max() / max(np.abs(oft).max(), 1.0)
    print("forces: %d spheres, max relative difference %.2e" % (len(oft), df))
    assert df < 1e-11
    return dv, dm


def test_flume_full_size_fp64():
    dv, dm = compare_fp64(I.flume(seed=2), 5)
    print("1536x40x192, 5 steps: max |du| %.2e, max |dm| %.2e" % (dv, dm))
    assert dv < 1e-13 and dm < 1e-12


@functools.lru_cache(maxsize=1)
def large_flume():
    return I.flume(nx=3072, ny=80, nz=256, seed=5)


def test_large_flume_full_size_fp64():
    dv, dm = compare_fp64(large_flume(), 2)
    print("3072x80x256, 2 steps: max |du| %.2e, max |dm| %.2e" % (dv, dm))
    assert dv < 1e-13 and dm < 1e-12


def test_large_flume_bed_particles_fp64():
    """The particle step on the large flume's 9,210 spheres (lowest layer
    fixed), 2 lattice steps of 10 sub-steps under gravity with lubrication,
    against the oracle's all-pairs evaluation."""
    w = large_flume()
    c, r = w.centre, w.radius
    fixed = (c[:, 2] < c[:, 2].min() + 2.0).astype(np.uint8)
    kw = dict(density=2.55, restitution=0.97, collision_time=40.0, poisson=0.22, friction=0.5,
              viscosity=1e-3, lub_cut=0.6, lub_min=1e-3, accel=(0, 0, -1e-4), dt=1.0, substeps=10)
    g = F().Dem(w.shape, c, r, None, None, fixed, skin=1.0, **kw)
    o = O.OracleDem(w.shape, c, r, None, None, fixed, **kw)
    g.step(None, n=2)
    o.step(None, n=2)
    worst = 0.0
    for a, b in zip(g.state(), o.state()):
        worst = max(worst, np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))
    print("3072x80x256 bed, %d spheres: max relative difference %.3e" % (len(r), worst))
    assert worst <= 1e-12
    g.destroy()


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_flume_full_size_properties(prec):
    f = F()
    w = I.flume(seed=2)
    g = f.lattice_from_workload(w, prec)
    M0 = g.total_mass()
    g.step(200)
    M1 = g.total_mass()
    fl = g.read_fields([f.FIELD_TYPE, f.FIELD_FILL, f.FIELD_NORMAL])
    g.destroy()
    assert abs(M1 - M0) <= 1e-12 * M0
    t = fl[f.FIELD_TYPE]
    liq, gas = t == f.LIQUID, t == f.GAS
    nz = t.shape[0]
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                sh = np.roll(np.roll(gas, dy, 1), dx, 2)
                if dz == 1:
                    sh = np.concatenate([np.zeros_like(sh[:1]), sh[:-1]], 0)
                elif dz == -1:
                    sh = np.concatenate([sh[1:], np.zeros_like(sh[:1])], 0)
                assert not np.any(liq & sh), (dz, dy, dx)
    itf = t == f.INTERFACE
    assert np.all(np.isfinite(fl[f.FIELD_FILL][itf]))
    nn = np.linalg.norm(fl[f.FIELD_NORMAL][:, itf], axis=0)
    assert np.all((np.abs(nn - 1.0) < 1e-5) | (nn == 0.0))
    assert nz == 192
