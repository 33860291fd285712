"""The GPU build of the kernels against the same kernel sources built for
the CPU (tests/hostemu), cell by cell, in every storage form.

Both run identical source; only the compilers differ (and the GPU may fuse
multiply-adds), so the cell types must agree exactly and the fields to a
few roundings of the storage form.  A difference of order one is the GPU
compiler's: this check caught a build of the interface kernel in which the
mass loaded at the start reached the final sum only in the lanes of one
divergent branch (the others added the flux to a stale register).  Cases:
tiny lattices with and without the Galilean correction, the film with its
crests at the top wall, and the splash (all free-surface variants).
"""
import dataclasses
import os
import sys

import numpy as np
import pytest

from paper_2301_10674_amd import inputs as I

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "hostemu"))
import emu  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-13, "fp32": 2e-6, "fp16": 2e-3}


def F():
    from paper_2301_10674_amd import fsl
    return fsl


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


CASES = {
    "tiny333": (lambda: tiny((3, 3, 3), 1.6), {}, 20),
    "tiny633_galilean": (lambda: tiny((6, 3, 3), 1.6), dict(galilean=True), 20),
    "tiny335_galilean": (lambda: tiny((3, 3, 5), 2.6), dict(galilean=True), 20),
    "lid": (lambda: I.film_with_surface_spheres(nz=22, sigma=1e-3), {}, 6),
    "splash_variants": (lambda: I.splash(shape=(24, 16, 20)),
                        dict(flux_modifiers=True, normal_excess=True, csf_curvature=True), 6),
}


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_gpu_build_matches_cpu_build(case, prec):
    f = F()
    make, kw, steps = CASES[case]
    w = make()
    g = f.lattice_from_workload(w, prec, **kw)
    e = emu.EmuLattice(w, prec, **kw)
    for k in range(2):
        g.step(steps // 2)
        e.step(steps // 2)
        t = e.read(f.FIELD_TYPE)
        assert np.array_equal(g.read(f.FIELD_TYPE), t), (case, prec, k)
        fl = (t == f.LIQUID) | (t == f.INTERFACE)
        dm = np.abs(g.read(f.FIELD_MASS) - e.read(f.FIELD_MASS))[fl].max()
        dp = np.abs(g.read(f.FIELD_PDF) - e.read(f.FIELD_PDF))[:, fl].max()
        print(case, prec, "after %d steps: max |dm| %.2e, max |df| %.2e" % ((k + 1) * (steps // 2), dm, dp))
        assert dm <= TOL[prec] and dp <= TOL[prec], (case, prec, dm, dp)
    assert np.array_equal(g.counters()[:7], e.counters()[:7])
    g.destroy()
    e.destroy()
