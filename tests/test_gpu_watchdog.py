"""GPU tests of the step watchdog (FslParams.check_every).

On a check step the dense and interface kernels reduce the total mass and
the density range per block, a one-block kernel combines them in a fixed
order with the excess-mass pool, and the host raises FSL_ERR_UNSTABLE for a
non-finite mass, a fluid density outside [0.5, 1.5], or a mass that drifted
by more than 1e-10 relative from the exact total after set-up.

* a healthy run checked on every step passes, and the watchdog's mass (the
  mass before each step's conversions, which only move mass) equals the
  exact fixed-order total to 1e-13 relative;
* a liquid region created at density 1.6 trips the density check on the
  first checked step, and the state stays readable;
* mass created by a poke into the stored PDFs (the current PDFs are the
  first PDF array of the workspace before the first step; f_i of cell
  (x, y, z) is element (27 (y + ny z) + i) nx + x) trips the drift check on
  the next checked step, not before;
* a flow compressed beyond density 1.5 by strong gravity is stopped with
  FSL_ERR_UNSTABLE on the first checked step past it.
"""
import numpy as np
import pytest

from paper_2301_10674_amd import inputs as I

pytestmark = pytest.mark.gpu


def F():
    from paper_2301_10674_amd import fsl
    return fsl


def test_healthy_run_passes_every_check():
    f = F()
    w = I.channel_film()
    g = f.lattice_from_workload(w, "fp64", check_every=1)
    for _ in range(4):
        g.step(5)
        wd = g.watchdog()
        m = g.total_mass()
        assert abs(wd["mass"] - m) <= 1e-13 * m, (wd, m)
        assert abs(wd["mass_ref"] - m) <= 1e-12 * m
        assert wd["cells_out"] == 0 and 0.99 < wd["rho_min"] <= wd["rho_max"] < 1.01
    g.destroy()


def test_total_mass_after_steps_matches_oracle():
    """Right after steps the total mass comes from the last step's block
    partials (and the pool before its conversions); it equals the oracle's
    exact total, and the exact recomputation of the set-up state."""
    from oracle import oracle as O

    f = F()
    w = I.film_with_surface_spheres(sigma=1e-3)
    o = O.OracleLattice(w.shape, w.omega, accel=w.accel, sigma=w.sigma, rho_gas=w.rho_gas,
                        conv_eps=w.conv_eps, fill=w.fill, rho=w.rho, vel=w.vel)
    o.set_particles(w.centre, w.radius, w.sphere_vel, w.sphere_angvel)
    g = f.lattice_from_workload(w, "fp64")
    m0 = g.total_mass()                     # exact pass (nothing stepped yet)
    assert abs(m0 - o.total_mass()) <= 1e-13 * m0
    for k in range(3):
        g.step(7)
        o.step(7)
        m = g.total_mass()
        assert abs(m - o.total_mass()) <= 1e-13 * m, (k, m, o.total_mass())
        assert abs(m - m0) <= 1e-13 * m0
    g.destroy()


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_total_mass_after_steps_is_conserved(prec):
    f = F()
    w = I.splash(shape=(24, 16, 20))
    g = f.lattice_from_workload(w, prec)
    m0 = g.total_mass()
    g.step(30)
    m1 = g.total_mass()
    assert abs(m1 - m0) <= 1e-12 * m0, (m0, m1)
    g.destroy()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16"])
def test_density_out_of_range_is_caught(prec):
    f = F()
    w = I.channel_film()
    rho = w.rho.copy()
    rho[2:6, :, 20:30] = 1.6            # a dense block inside the liquid
    import dataclasses
    w = dataclasses.replace(w, rho=rho)
    g = f.lattice_from_workload(w, prec, check_every=2)
    g.step(1)                             # not a check step
    with pytest.raises(f.FslError) as e:
        g.step(1)
    assert "status 5" in str(e.value) and "density" in str(e.value)
    wd = g.watchdog()
    assert wd["cells_out"] > 20 and wd["rho_max"] > 1.5
    assert np.isfinite(g.read(f.FIELD_RHO)).all()    # still readable
    g.destroy()


def test_mass_drift_is_caught():
    f = F()
    w = I.channel_film()
    g = f.lattice_from_workload(w, "fp64", check_every=3)
    nx, ny, nz = w.shape
    N = nx * ny * nz
    t = g.read(f.FIELD_TYPE)
    z, y, x = 12, 4, 40
    assert t[z, y, x] == f.LIQUID and (t[z - 1:z + 2, y - 1:y + 2, x - 1:x + 2] == f.LIQUID).all()
    pdf = g.workspace[:27 * N * 8].view(dtype=__import__("torch").float64)
    i = 1 + 3 * 1 + 9 * 2                 # c = (0, 0, +1), pulled by the cell above
    pdf[(27 * (y + ny * z) + i) * nx + x] += 1e-4
    g.step(2)                             # no check yet
    with pytest.raises(f.FslError) as e:
        g.step(1)
    assert "status 5" in str(e.value) and "drifted" in str(e.value)
    wd = g.watchdog()
    assert abs((wd["mass"] - wd["mass_ref"]) - 1e-4) < 1e-9
    g.destroy()


def test_flow_leaving_the_weakly_compressible_range_is_stopped():
    """Gravity of 0.03 on the film compresses the liquid column beyond
    density 1.5 within about ten steps; the check on every step stops the
    run there."""
    f = F()
    import dataclasses
    w = dataclasses.replace(I.channel_film(), accel=(0.0, 0.0, -0.03))
    g = f.lattice_from_workload(w, "fp32", check_every=1)
    with pytest.raises(f.FslError) as e:
        g.step(100)
    assert "status 5" in str(e.value) and "density" in str(e.value)
    info = g.info()
    assert 3 <= info[0] <= 40, info
    g.destroy()
