"""GPU parity: the HIP path (through the C-ABI) against the FP64 CPU oracle.

Both sides start from the same seeded inputs (``paper_2301_10674_amd.inputs``)
and share no other code.  The FP64 form must match element by element to
rounding level; FP32 and FP16 storage must stay within the velocity error
targets (relative L2 1e-5 and 1e-3) and conserve mass to 1e-12.
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
    if len(w.radius):
        L.set_particles(w.centre, w.radius, w.sphere_vel, w.sphere_angvel)
    return L


def gpu_fields(g):
    f = F()
    return g.read_fields([f.FIELD_TYPE, f.FIELD_MASS, f.FIELD_FILL, f.FIELD_RHO, f.FIELD_VEL,
                          f.FIELD_PDF, f.FIELD_NORMAL, f.FIELD_CURV, f.FIELD_OWNER])


def oracle_fields(o):
    f = F()
    return {f.FIELD_TYPE: o.read(O.F_TYPE), f.FIELD_MASS: o.read(O.F_MASS),
            f.FIELD_FILL: o.read(O.F_FILL), f.FIELD_RHO: o.read(O.F_RHO),
            f.FIELD_VEL: o.read(O.F_VEL), f.FIELD_PDF: o.read(O.F_PDF),
            f.FIELD_NORMAL: o.read(O.F_NORMAL), f.FIELD_CURV: o.read(O.F_CURV),
            f.FIELD_OWNER: o.read(O.F_OWNER)}


def assert_fp64_parity(gf, of, tol=1e-12, label=""):
    f = F()
    t = of[f.FIELD_TYPE]
    assert np.array_equal(gf[f.FIELD_TYPE], t), label + ": cell types differ"
    assert np.array_equal(gf[f.FIELD_OWNER], of[f.FIELD_OWNER]), label + ": owners differ"
    fluid = (t == O.LIQUID) | (t == O.INTERFACE)
    itf = t == O.INTERFACE
    worst = {}
    worst["pdf"] = np.abs(gf[f.FIELD_PDF][:, fluid] - of[f.FIELD_PDF][:, fluid]).max(initial=0)
    worst["mass"] = np.abs(gf[f.FIELD_MASS][fluid] - of[f.FIELD_MASS][fluid]).max(initial=0)
    worst["rho"] = np.abs(gf[f.FIELD_RHO][fluid] - of[f.FIELD_RHO][fluid]).max(initial=0)
    worst["fill"] = np.abs(gf[f.FIELD_FILL][itf] - of[f.FIELD_FILL][itf]).max(initial=0)
    worst["vel"] = np.abs(gf[f.FIELD_VEL][:, fluid] - of[f.FIELD_VEL][:, fluid]).max(initial=0)
    worst["normal"] = np.abs(gf[f.FIELD_NORMAL][:, itf] - of[f.FIELD_NORMAL][:, itf]).max(initial=0)
    worst["curv"] = np.abs(gf[f.FIELD_CURV][itf] - of[f.FIELD_CURV][itf]).max(initial=0)
    bad = {k: v for k, v in worst.items() if not v <= tol}
    assert not bad, "%s: %s" % (label, worst)
    return worst


def velocity_rel_l2(gf, of):
    f = F()
    both = ((gf[f.FIELD_TYPE] == O.LIQUID) | (gf[f.FIELD_TYPE] == O.INTERFACE)) & \
           ((of[f.FIELD_TYPE] == O.LIQUID) | (of[f.FIELD_TYPE] == O.INTERFACE))
    du = gf[f.FIELD_VEL][:, both] - of[f.FIELD_VEL][:, both]
    return np.sqrt((du ** 2).sum() / (of[f.FIELD_VEL][:, both] ** 2).sum())


# ------------------------------------------------------------------ FP64 parity
def test_initial_state_matches():
    w = I.channel_film()
    g = F().lattice_from_workload(w, "fp64")
    o = oracle_from(w)
    assert_fp64_parity(gpu_fields(g), oracle_fields(o), 1e-14, "init")
    # both sums are FP64 over ~1e4 cells in different orders
    assert abs(g.total_mass() - o.total_mass()) < 1e-14 * o.total_mass()


@pytest.mark.parametrize("steps", [1, 5])
def test_channel_film_first_steps_fp64(steps):
    w = I.channel_film()
    g = F().lattice_from_workload(w, "fp64")
    o = oracle_from(w)
    g.step(steps)
    o.step(steps)
    assert_fp64_parity(gpu_fields(g), oracle_fields(o), 1e-13, "step %d" % steps)


def test_channel_film_200_steps_fp64():
    w = I.channel_film()
    g = F().lattice_from_workload(w, "fp64")
    o = oracle_from(w)
    M0 = o.total_mass()
    assert abs(g.total_mass() - M0) < 1e-14 * M0
    for k in range(4):
        g.step(50)
        o.step(50)
        assert_fp64_parity(gpu_fields(g), oracle_fields(o), 1e-12, "after %d steps" % (50 * (k + 1)))
    assert np.array_equal(g.counters()[:7], o.counters()[:7])
    assert abs(g.total_mass() - M0) <= 1e-12 * M0


def test_moving_rotating_spheres_fp64():
    nx, ny, nz = 12, 10, 12
    rng = np.random.default_rng(1)
    vel = 0.01 * rng.standard_normal((3, nz, ny, nx))
    w = I.Workload(name="box", shape=(nx, ny, nz), omega=1.7, accel=(1e-5, 2e-6, -3e-6),
                   sigma=0.0, fill=np.ones((nz, ny, nx)), rho=1 + 0.01 * rng.standard_normal((nz, ny, nx)),
                   vel=vel, centre=np.array([[3.0, 4.0, 5.0], [8.5, 7.2, 6.1], [11.7, 0.3, 2.0]]),
                   radius=np.array([2.5, 3.0, 2.2]),
                   sphere_vel=np.array([[1e-3, 0, -1e-3], [0, 2e-3, 0], [5e-4, 5e-4, 5e-4]]),
                   sphere_angvel=np.array([[0, 0, 1e-3], [1e-3, 0, 0], [2e-4, -3e-4, 1e-4]]))
    g = F().lattice_from_workload(w, "fp64")
    o = oracle_from(w)
    g.step(30)
    o.step(30)
    assert_fp64_parity(gpu_fields(g), oracle_fields(o), 1e-13, "spheres")


@pytest.mark.parametrize("shape,h", [((300, 3, 7), 3.4), ((3, 3, 3), 1.6), ((257, 5, 9), 5.0)])
def test_ragged_and_tiny_lattices_fp64(shape, h):
    """Ragged x tails (300, 257 cells over 256-wide blocks), the smallest
    lattice, and a surface exactly on a cell face."""
    nx, ny, nz = shape
    xc = np.arange(nx) + 0.5
    hh = h + 0.7 * np.sin(2 * np.pi * xc / nx)
    fill = I.height_fill(shape, np.broadcast_to(hh[None, :], (ny, nx)))
    rng = np.random.default_rng(5)
    w = I.Workload(name="rag", shape=shape, omega=1.3, accel=(1e-4, 0, -1e-4), sigma=1e-3,
                   fill=fill, rho=np.ones((nz, ny, nx)), vel=0.01 * rng.standard_normal((3, nz, ny, nx)),
                   centre=np.zeros((0, 3)), radius=np.zeros(0), sphere_vel=np.zeros((0, 3)),
                   sphere_angvel=np.zeros((0, 3)))
    g = F().lattice_from_workload(w, "fp64")
    o = oracle_from(w)
    M0 = o.total_mass()
    g.step(20)
    o.step(20)
    assert_fp64_parity(gpu_fields(g), oracle_fields(o), 1e-12, str(shape))
    assert abs(g.total_mass() - M0) <= 1e-12 * M0


def test_all_liquid_has_empty_interface_list():
    nx, ny, nz = 64, 4, 6
    w = I.Workload(name="liq", shape=(nx, ny, nz), omega=1.5, accel=(1e-5, 0, 0), sigma=0.0,
                   fill=np.ones((nz, ny, nx)), rho=np.ones((nz, ny, nx)), vel=np.zeros((3, nz, ny, nx)),
                   centre=np.zeros((0, 3)), radius=np.zeros(0), sphere_vel=np.zeros((0, 3)),
                   sphere_angvel=np.zeros((0, 3)))
    g = F().lattice_from_workload(w, "fp64")
    o = oracle_from(w)
    assert g.info()[1] == 0
    g.step(10)
    o.step(10)
    assert_fp64_parity(gpu_fields(g), oracle_fields(o), 1e-13, "liquid box")


def test_flume_crop_fp64():
    w = I.flume(nx=64, ny=40, nz=96, seed=7)
    g = F().lattice_from_workload(w, "fp64")
    o = oracle_from(w)
    M0 = o.total_mass()
    g.step(10)
    o.step(10)
    assert_fp64_parity(gpu_fields(g), oracle_fields(o), 1e-12, "flume crop")
    assert abs(g.total_mass() - M0) <= 1e-12 * M0


# ------------------------------------------------------------------ reduced precision
@pytest.mark.parametrize("prec,target", [("fp32", 1e-5), ("fp16", 1e-3)])
def test_channel_film_reduced_precision(prec, target):
    w = I.channel_film()
    g = F().lattice_from_workload(w, prec)
    o = oracle_from(w)
    M0 = o.total_mass()
    g.step(200)
    o.step(200)
    gf, of = gpu_fields(g), oracle_fields(o)
    err = velocity_rel_l2(gf, of)
    assert err <= target, err
    assert abs(g.total_mass() - M0) <= 1e-12 * M0
    flips = (gf[F().FIELD_TYPE] != of[F().FIELD_TYPE]).sum()
    assert flips <= 0.01 * w.ncells


def test_determinism_fp32():
    w = I.channel_film()
    res = []
    for _ in range(2):
        g = F().lattice_from_workload(w, "fp32")
        g.step(50)
        res.append(gpu_fields(g))
    for k in res[0]:
        assert np.array_equal(res[0][k], res[1][k]), k


@pytest.mark.parametrize("case,prec", [("film", "fp64"), ("splash", "fp32")])
def test_launch_geometry_does_not_change_results(case, prec):
    """The same lattice stepped with the automatic launch geometry and with 8
    and 24 workgroups for the dense pass and the interface-list kernels
    (each workgroup then walks many more row segments and list entries):
    every cell's state is bit-identical; the total mass, a sum of
    per-workgroup partials, agrees to rounding."""
    w = I.film_with_surface_spheres(sigma=1e-3) if case == "film" else I.splash(shape=(24, 16, 20))
    res, mass = [], []
    for gb in (0, 8, 24):
        g = F().lattice_from_workload(w, prec, grid_blocks=gb)
        g.step(40)
        res.append(gpu_fields(g))
        mass.append(g.total_mass())
        g.destroy()
    for r in res[1:]:
        for k in res[0]:
            assert np.array_equal(res[0][k], r[k]), k
    assert max(abs(m - mass[0]) for m in mass) <= 1e-14 * mass[0], mass


# ------------------------------------------------------------------ error paths
def test_argument_and_state_errors():
    f = F()
    w = I.channel_film()
    with pytest.raises(f.FslError) as e:
        f.Lattice(f.make_params(w.shape, "fp64", omega=2.0), w.fill, w.rho)
    assert e.value.status == f.FSL_ERR_ARG
    bad = w.rho.copy()
    bad[3, 2, 1] = np.nan
    with pytest.raises(f.FslError) as e:
        f.Lattice(f.make_params(w.shape, "fp64", omega=1.9), w.fill, bad)
    assert e.value.status == f.FSL_ERR_ARG
    g = f.lattice_from_workload(w, "fp64")
    g.step(1)
    with pytest.raises(f.FslError) as e:
        g.set_particles(w.centre + 1.0, w.radius)
    assert e.value.status == f.FSL_ERR_STATE
    # velocities alone may change
    g.set_particles(w.centre, w.radius, vel=np.full((len(w.radius), 3), 1e-4))
    with pytest.raises(f.FslError) as e:
        g.set_particles(w.centre, np.full(len(w.radius), 2.9))
    assert e.value.status == f.FSL_ERR_STATE
    with pytest.raises(f.FslError) as e:
        g.set_particles(w.centre, np.full(len(w.radius), 5.0))   # r >= ny/2
    assert e.value.status == f.FSL_ERR_ARG
