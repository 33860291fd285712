"""GPU parity of the particle motion (fsl_dem_*) and of the coupled
fluid-particle step against the FP64 oracle, through the C-ABI.

* A cluster of 60 spheres (radii 2.5-4, some overlapping, some fixed)
  under gravity, a constant hydrodynamic load, collisions with friction,
  walls and lubrication, 40 lattice steps of 10 sub-steps: positions,
  velocities and spins agree to 1e-12 of their scale (both sides evaluate
  each pair in the same order with the same roundings, except that the
  logarithm of the tangential lubrication may round differently); the
  bedload rate of Eq. (1) to 1e-13.
* The flume bed (1,848 spheres of the benchmark, the lowest layer fixed)
  settling under gravity for 5 steps: the same bound.
* Coupled steps (fluid step, momentum-exchange forces, particle sub-steps,
  remap) of three spheres falling through liquid onto the bottom wall:
  lattice fields and particle states agree with the oracle run through the
  same sequence.
* Error paths: too many partners, a sphere faster than the skin allows.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2301_10674_amd import inputs as I

from test_gpu_parity import assert_fp64_parity, gpu_fields, oracle_fields

pytestmark = pytest.mark.gpu

KW = dict(density=2.55, restitution=0.97, collision_time=40.0, poisson=0.22, friction=0.5)


def F():
    from paper_2301_10674_amd import fsl
    return fsl


def compare(g, o, rel=1e-12, label=""):
    worst = 0.0
    for a, b, name in zip(g, o, ("centre", "vel", "angvel")):
        scale = max(np.abs(b).max(), 1e-30)
        err = np.abs(a - b).max() / scale
        worst = max(worst, err)
        assert err <= rel, (label, name, err)
    return worst


def test_cluster_fp64():
    box = (48, 36, 30)
    c, r, v, w, fixed = I.sphere_cluster(box)
    rng = np.random.default_rng(2)
    hydro = 1e-3 * rng.standard_normal((len(r), 6))
    kw = dict(KW, viscosity=0.05, lub_cut=0.6, lub_min=1e-3, accel=(0, 0, -5e-4), dt=1.0, substeps=10)
    g = F().Dem(box, c, r, v, w, fixed, skin=1.0, **kw)
    o = O.OracleDem(box, c, r, v, w, fixed, **kw)
    for k in range(4):
        g.step(hydro, n=10)
        o.step(hydro, n=10)
        err = compare(g.state(), o.state(), 1e-12, "after %d steps" % (10 * (k + 1)))
        print("after %d steps: max relative difference %.3e" % (10 * (k + 1), err))
    x, vv, ww = g.state()
    qg, qo = g.bedload(), o.bedload()
    print("bedload rate %.6e (oracle %.6e)" % (qg, qo))
    assert abs(qg - qo) <= 1e-13 * max(abs(qo), 1e-30) and abs(qo) > 0
    assert np.abs(vv - v).max() > 1e-3            # collisions happened
    assert np.array_equal(x[fixed == 1], c[fixed == 1])
    g.destroy()


def test_flume_bed_settling_fp64():
    w = I.flume(seed=2)
    c, r = w.centre, w.radius
    fixed = (c[:, 2] < c[:, 2].min() + 2.0).astype(np.uint8)
    kw = dict(KW, viscosity=1e-3, lub_cut=0.6, lub_min=1e-3, accel=(0, 0, -1e-4), dt=1.0, substeps=10)
    g = F().Dem(w.shape, c, r, None, None, fixed, skin=1.0, **kw)
    o = O.OracleDem(w.shape, c, r, None, None, fixed, **kw)
    g.step(None, n=5)
    o.step(None, n=5)
    err = compare(g.state(), o.state(), 1e-12, "flume bed")
    print("flume bed, %d spheres (%d fixed): max relative difference %.3e" % (len(r), fixed.sum(), err))
    g.destroy()


def test_coupled_settling_fp64():
    w = I.settling_box()
    f = F()
    from paper_2301_10674_amd.couple import Coupled
    kw = dict(KW, viscosity=(1 / w.omega - 0.5) / 3, lub_cut=0.6, lub_min=1e-3, accel=w.accel,
              dt=1.0, substeps=10)
    lat = f.lattice_from_workload(w, "fp64")
    dem = f.Dem(w.shape, w.centre, w.radius, w.sphere_vel, w.sphere_angvel, None, skin=1.0, **kw)
    run = Coupled(lat, dem)
    o = O.OracleLattice(w.shape, w.omega, accel=w.accel, sigma=w.sigma, rho_gas=w.rho_gas,
                        conv_eps=w.conv_eps, fill=w.fill, rho=w.rho, vel=w.vel)
    o.set_particles(w.centre, w.radius, w.sphere_vel, w.sphere_angvel)
    od = O.OracleDem(w.shape, w.centre, w.radius, w.sphere_vel, w.sphere_angvel, None, **kw)
    M0 = o.total_mass()
    for k in range(3):
        run.step(10)
        for _ in range(10):
            o.step(1)
            od.step(o.particle_forces())
            o.move_particles(*od.state())
        err = compare(dem.state(), od.state(), 1e-11, "coupled, %d steps" % (10 * (k + 1)))
        assert_fp64_parity(gpu_fields(lat), oracle_fields(o), 1e-11, "coupled, %d steps" % (10 * (k + 1)))
        print("coupled, %d steps: particles max relative difference %.3e" % (10 * (k + 1), err))
    x, v, _ = dem.state()
    assert x[0, 2] < 3.3 and v[:, 2].max() > -0.02      # the spheres were slowed / stopped
    assert abs(lat.total_mass() - M0) <= 1e-12 * M0
    lat.destroy()
    dem.destroy()


def test_collision_across_the_periodic_seam_fp64():
    kw = dict(KW, dt=0.05, substeps=1)
    c = [[34.9, 20, 20], [5.1, 20.3, 19.8]]
    v = [[0.02, 0.001, 0], [-0.02, 0, 0.001]]
    w = [[0, 0, 0.003], [0.002, 0, 0]]
    g = F().Dem((40, 40, 40), c, [5.0, 5.0], v, w, None, skin=1.0, **kw)
    o = O.OracleDem((40, 40, 40), c, [5.0, 5.0], v, w, None, **kw)
    g.step(None, n=2000)
    o.step(None, n=2000)
    err = compare(g.state(), o.state(), 1e-12, "seam")
    x, vv, _ = g.state()
    assert vv[1, 0] > 0.0 and (x[:, 0] >= 0).all() and (x[:, 0] < 40).all()
    print("collision across x = 0: max relative difference %.3e" % err)
    g.destroy()


def test_coupled_device_path_matches_host_path():
    """The coupled step through device tensors (forces, particle state and
    the remap's input never leave the GPU) gives the same bits as the step
    through host arrays; a non-finite device input is rejected before
    anything changes."""
    import torch

    from paper_2301_10674_amd.couple import Coupled
    f = F()
    w = I.settling_box()
    kw = dict(KW, viscosity=(1 / w.omega - 0.5) / 3, lub_cut=0.6, lub_min=1e-3, accel=w.accel,
              dt=1.0, substeps=10)
    res = []
    for host in (False, True):
        lat = f.lattice_from_workload(w, "fp64")
        dem = f.Dem(w.shape, w.centre, w.radius, w.sphere_vel, w.sphere_angvel, None, skin=1.0, **kw)
        run = Coupled(lat, dem)
        (run.step_host if host else run.step)(15)
        res.append((dem.state(), lat.read_fields([f.FIELD_PDF, f.FIELD_MASS, f.FIELD_OWNER])))
        if not host:
            before = lat.read_fields([f.FIELD_TYPE, f.FIELD_OWNER])
            c, v, a = dem.state_device()
            c[1, 2] = float("nan")
            with pytest.raises(f.FslError) as e:
                lat.move_particles_device(c, v, a)
            assert e.value.status == f.FSL_ERR_ARG
            after = lat.read_fields([f.FIELD_TYPE, f.FIELD_OWNER])
            for k in before:
                assert np.array_equal(before[k], after[k])
            torch.cuda.synchronize()
        lat.destroy()
        dem.destroy()
    (sa, fa), (sb, fb) = res
    for a, b in zip(sa, sb):
        assert np.array_equal(a, b)
    for k in fa:
        assert np.array_equal(fa[k], fb[k]), k


@pytest.mark.parametrize("case", ["single", "between_walls"])
def test_small_cases_fp64(case):
    """One free sphere falling onto the bottom wall and bouncing; a sphere
    that touches both walls of a box only slightly taller than it is wide
    (both wall contacts at once)."""
    if case == "single":
        box, c, r, v = (20, 20, 20), [[10.0, 10.0, 6.0]], [5.0], [[0.003, -0.002, -0.03]]
    else:
        box, c, r, v = (20, 20, 10), [[10.0, 10.0, 5.0]], [5.05], [[0.01, 0.0, 0.002]]
    kw = dict(KW, viscosity=0.02, lub_cut=0.6, lub_min=1e-3, accel=(0, 0, -1e-4), dt=1.0, substeps=10)
    g = F().Dem(box, c, r, v, [[0, 0.001, 0]], None, skin=1.0, **kw)
    o = O.OracleDem(box, c, r, v, [[0, 0.001, 0]], None, **kw)
    g.step(None, n=100)
    o.step(None, n=100)
    err = compare(g.state(), o.state(), 1e-12, case)
    print(case, "max relative difference %.3e" % err)
    g.destroy()


def test_error_paths():
    f = F()
    # 60 small spheres in a cube of side 0.8: every other sphere is within
    # reach (r_i + r_j + skin = 1.4 > the cube's diagonal), 59 > 32 partners
    rng = np.random.default_rng(0)
    c = 10 + rng.uniform(0, 0.8, (60, 3))
    g = f.Dem((20, 20, 20), c, np.full(60, 0.2), skin=1.0)
    with pytest.raises(f.FslError) as e:
        g.step()
    assert e.value.status == f.FSL_ERR_NOMEM
    g.destroy()
    # a sphere crossing more than half the skin in one step
    g = f.Dem((50, 50, 50), [[25, 25, 25]], [2.0], vel=[[0.8, 0, 0]], skin=1.0)
    with pytest.raises(f.FslError) as e:
        g.step()
    assert e.value.status == f.FSL_ERR_UNSTABLE
    x, _, _ = g.state()
    assert abs(x[0, 0] - 25.8) < 1e-12
    g.destroy()
