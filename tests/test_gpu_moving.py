"""GPU parity of moving spheres (fsl_move_particles) against the oracle,
through the C-ABI.

* FP64, a box with a free surface and two spheres: random moves (some that
  remap cells, some too small to change any cell) each followed by a few
  steps; cell types and owners identical, PDFs, masses and velocities of
  fluid cells to 1e-12, total mass exact;
* a two-cell shift through liquid (uncovered cells typed in several
  rounds);
* FP32 and FP16 storage: the total mass stays exact over moves and steps;
* argument and state errors.
"""
import numpy as np
import pytest

from oracle import oracle as O

pytestmark = pytest.mark.gpu


def F():
    from paper_2301_10674_amd import fsl
    return fsl


def film(shape, h):
    nx, ny, nz = shape
    z = np.arange(nz)[:, None, None] + np.zeros((nz, ny, nx))
    return np.clip(h - z, 0.0, 1.0)


def pair(shape, fill, centre, radius, prec="fp64", accel=(1e-5, 0.0, -1e-5), omega=1.5):
    f = F()
    nx, ny, nz = shape
    p = f.make_params(shape=shape, precision=prec, omega=omega, accel=accel, sigma=0.0,
                      rho_gas=1.0, conv_eps=1e-3, check_every=0)
    g = f.Lattice(p, fill, np.ones((nz, ny, nx)))
    g.set_particles(centre, radius)
    o = O.OracleLattice(shape, omega, accel=accel, fill=fill, rho=np.ones((nz, ny, nx)), conv_eps=1e-3)
    o.set_particles(centre, radius)
    return g, o


def compare(g, o, label):
    f = F()
    gf = g.read_fields([f.FIELD_TYPE, f.FIELD_OWNER, f.FIELD_PDF, f.FIELD_MASS, f.FIELD_VEL])
    t = o.read(O.F_TYPE)
    assert np.array_equal(gf[f.FIELD_TYPE], t), label + ": types"
    assert np.array_equal(gf[f.FIELD_OWNER], o.read(O.F_OWNER)), label + ": owners"
    fl = (t == O.LIQUID) | (t == O.INTERFACE)
    worst = max(np.abs(gf[f.FIELD_PDF][:, fl] - o.read(O.F_PDF)[:, fl]).max(),
                np.abs(gf[f.FIELD_MASS][fl] - o.read(O.F_MASS)[fl]).max(),
                np.abs(gf[f.FIELD_VEL][:, fl] - o.read(O.F_VEL)[:, fl]).max())
    assert worst < 1e-12, (label, worst)
    # summation order differs (cells in blocks vs in sequence): rounding
    assert abs(g.total_mass() - o.total_mass()) <= 1e-13 * o.total_mass(), label


def test_random_moves_fp64():
    shape = (24, 12, 20)
    c = np.array([[6.0, 6.0, 5.0], [15.5, 4.2, 11.0]])
    g, o = pair(shape, film(shape, 12.3), c, [2.6, 2.2])
    M0 = o.total_mass()
    rng = np.random.default_rng(4)
    for k in range(10):
        step = rng.uniform(-0.7, 0.7, size=c.shape) if k % 3 else rng.uniform(-0.02, 0.02, size=c.shape)
        c = c + step
        c[:, 2] = np.clip(c[:, 2], 3.5, 15.0)
        v = rng.normal(0, 1e-3, size=c.shape)
        w = rng.normal(0, 1e-4, size=c.shape)
        g.move_particles(c, v, w)
        o.move_particles(c, v, w)
        compare(g, o, "move %d" % k)
        g.step(3)
        o.step(3)
        compare(g, o, "move %d + 3 steps" % k)
    assert abs(g.total_mass() - M0) <= 1e-12 * M0
    g.destroy()


def test_two_cell_shift_fp64():
    shape = (20, 16, 18)
    nx, ny, nz = shape
    c0 = np.array([[8.3, 7.6, 8.9]])
    g, o = pair(shape, np.ones((nz, ny, nx)), c0, [3.6], accel=(0.0, 0.0, 0.0))
    for a in (g, o):
        a.move_particles(c0 + np.array([2.0, -2.0, 1.0]), np.array([[2e-3, -1e-3, 5e-4]]),
                         np.array([[1e-4, 2e-4, -3e-4]]))
    compare(g, o, "shift")
    g.step(5)
    o.step(5)
    compare(g, o, "shift + 5 steps")
    g.destroy()


def test_far_moves_in_height_fp64():
    """Spheres jumping several cells up and down between moves, through
    liquid and into the gas above it: a remap clears and scans only the
    rows the spheres reach before or after the move, and those rows change
    from move to move.  Also the device move path, which reports the new
    rows from the device."""
    import torch
    shape = (22, 16, 28)
    c = np.array([[6.0, 8.0, 5.5], [15.0, 6.0, 6.0]])
    g, o = pair(shape, film(shape, 17.2), c, [2.4, 2.1])
    jumps = [np.array([[0.3, 0.0, 6.5], [0.0, -0.4, 0.0]]), np.array([[0.0, 0.2, 8.0], [0.5, 0.0, 9.0]]),
             np.array([[0.0, 0.0, -13.0], [0.0, 0.3, -7.5]]), np.array([[-0.4, 0.0, 3.0], [0.0, 0.0, 12.0]])]
    for k, dj in enumerate(jumps):
        c = c + dj
        v = np.full(c.shape, 1e-3)
        if k % 2:
            dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
            g.move_particles_device(dev(c), dev(v), None)
        else:
            g.move_particles(c, v)
        o.move_particles(c, v)
        compare(g, o, "jump %d" % k)
        g.step(3)
        o.step(3)
        compare(g, o, "jump %d + 3 steps" % k)
    g.destroy()


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_mass_exact_reduced_storage(prec):
    shape = (24, 12, 20)
    c = np.array([[6.0, 6.0, 5.0], [15.5, 4.2, 11.0]])
    g, _ = pair(shape, film(shape, 12.3), c, [2.6, 2.2], prec=prec)
    M0 = g.total_mass()
    rng = np.random.default_rng(7)
    for k in range(8):
        c = c + rng.uniform(-0.8, 0.8, size=c.shape)
        c[:, 2] = np.clip(c[:, 2], 3.5, 15.0)
        g.move_particles(c, rng.normal(0, 1e-3, size=c.shape))
        g.step(4)
        assert abs(g.total_mass() - M0) <= 1e-12 * M0
    g.destroy()


def test_errors():
    f = F()
    nx, ny, nz = 8, 8, 8
    p = f.make_params(shape=(nx, ny, nz), precision="fp64", omega=1.5)
    g = f.Lattice(p, np.ones((nz, ny, nx)), np.ones((nz, ny, nx)))
    c = np.array([[4.0, 4.0, 4.0]])
    assert f.lib().fsl_move_particles(g.h, f._dp(c.reshape(-1)), None, None) == f.FSL_ERR_STATE
    g.set_particles(c, [2.0])
    bad = np.array([np.nan, 4.0, 4.0])
    assert f.lib().fsl_move_particles(g.h, f._dp(bad), None, None) == f.FSL_ERR_ARG
    assert f.lib().fsl_move_particles(g.h, None, None, None) == f.FSL_ERR_ARG
    assert f.lib().fsl_move_particles(None, None, None, None) == f.FSL_ERR_STATE
    g.destroy()
