"""Pins of the oracle's interface geometry (normal and curvature).

Section 2.1 puts the local curvature kappa of the free surface into the
Laplace pressure 2 sigma kappa; the oracle estimates the normal with the
Parker-Youngs weights and kappa as the mean curvature from the finite-
difference Hessian of the same 3x3x3 fill stencil.  Both are exact for a
quadratic fill field, which gives a closed-form pin:
    phi = a + b.x + x.A.x/2  ->  grad = b, Hessian = A,
    n = -b/|b|, kappa = -(tr A - b^.A.b^) / (2 |b|).
The variant curvature (half the divergence of corner normals, Brackbill et
al. 1992) is pinned by planes (zero), spheres and cylinders (1/R and
1/(2R), second-order convergence), the complement field (opposite sign)
and the 48 symmetries of the cube.
"""
import numpy as np

from oracle import oracle as O

C, _ = O.velocities()


def stencil(fun):
    return np.array([fun(C[i].astype(float)) for i in range(27)])


def test_quadratic_field_is_exact():
    rng = np.random.default_rng(3)
    for _ in range(50):
        b = rng.standard_normal(3) * 0.05
        A = rng.standard_normal((3, 3)) * 0.01
        A = 0.5 * (A + A.T)
        a = 0.5
        phi = stencil(lambda x: a + b @ x + 0.5 * x @ A @ x)
        assert phi.min() > 0 and phi.max() < 1
        n, k = O.normal_curvature(phi)
        bn = np.linalg.norm(b)
        bh = b / bn
        assert np.max(np.abs(n + bh)) < 1e-14
        kex = -(np.trace(A) - bh @ A @ bh) / (2 * bn)
        assert abs(k - kex) < 1e-13 * max(1.0, abs(kex))


def test_planes_have_zero_curvature_and_exact_normal():
    rng = np.random.default_rng(4)
    for _ in range(50):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        phi = stencil(lambda x: 0.5 - 0.1 * d @ x)
        n, k = O.normal_curvature(phi)
        assert np.max(np.abs(n - d)) < 1e-14
        assert abs(k) < 1e-13


def test_sphere_field_gives_inverse_radius():
    """A smooth radial field phi(r) with the interface at radius R: the
    estimator returns a mean curvature close to 1/R (second-order stencil)."""
    for R in (8.0, 16.0, 32.0):
        centre = np.array([R, 0.3, -0.2])
        phi = stencil(lambda x: 0.5 - 0.1 * (np.linalg.norm(x - centre) - R))
        n, k = O.normal_curvature(phi)
        # liquid inside (phi decreases outwards), normal points away from the centre
        r = -centre / np.linalg.norm(centre)
        assert np.dot(n, r) > 0.999
        assert abs(k * R - 1.0) < 2.0 / R


def test_flat_stencil_gives_no_normal():
    n, k = O.normal_curvature(np.full(27, 0.3))
    assert np.all(n == 0.0) and k == 0.0


def test_lattice_geometry_of_flat_film():
    """On a lattice the stencil reads liquid as 1 and gas as 0; a flat film
    gives n = +z and kappa = 0 at every interface cell."""
    nx, ny, nz = 5, 4, 10
    h = 6.3
    k = np.arange(nz)[:, None, None]
    fill = np.clip(h - k, 0, 1) * np.ones((1, ny, nx))
    L = O.OracleLattice((nx, ny, nz), 1.0, fill=fill)
    t = L.read(O.F_TYPE)
    n = L.read(O.F_NORMAL)
    kap = L.read(O.F_CURV)
    itf = t == O.INTERFACE
    # cell 6 is partly filled; cell 5 touches only interface cells, so stays liquid
    assert itf.sum() == nx * ny and np.all(t[5] == O.LIQUID) and np.all(t[7] == O.GAS)
    top = itf & (k == 6)
    assert np.allclose(n[2][top], 1.0) and np.allclose(n[0][top], 0) and np.allclose(n[1][top], 0)
    assert np.max(np.abs(kap[itf])) < 1e-14


# ---- curvature from corner normals (Brackbill et al. 1992), a variant ----
def test_csf_planes_have_zero_curvature():
    rng = np.random.default_rng(14)
    for _ in range(50):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        phi = stencil(lambda x: 0.5 - 0.1 * d @ x)
        assert abs(O.csf_curvature(phi)) < 1e-14


def test_csf_sphere_and_cylinder():
    """Half the divergence of the unit normal: 1/R on a sphere, 1/(2R) on a
    cylinder, converging as the radius grows; a bubble (the complement
    field) has exactly the opposite curvature."""
    errs = []
    for R in (8.0, 16.0, 32.0, 64.0):
        centre = np.array([R, 0.3, -0.2])
        phi = stencil(lambda x: 0.5 - 0.1 * (np.linalg.norm(x - centre) - R))
        k = O.csf_curvature(phi)
        errs.append(abs(k * R - 1.0))
        assert abs(O.csf_curvature(1.0 - phi) + k) < 1e-14 * abs(k)
        axis = np.array([0.0, 0.0, 1.0])
        cyl = stencil(lambda x: 0.5 - 0.1 * (np.linalg.norm((x - centre) - ((x - centre) @ axis) * axis) - R))
        assert abs(O.csf_curvature(cyl) * 2 * R - 1.0) < 4.0 / R
    # second order: the error falls about fourfold per doubling of R
    assert errs[-1] < 2e-4 and all(b < 0.3 * a for a, b in zip(errs, errs[1:]))


def test_csf_is_invariant_under_the_cube_symmetries():
    rng = np.random.default_rng(15)
    phi = np.clip(rng.uniform(0, 1, 27), 0, 1)
    k0 = O.csf_curvature(phi)
    assert abs(k0) > 1e-3
    grid = phi.reshape(3, 3, 3)   # [z, y, x]
    for perm in ((0, 2, 1), (1, 0, 2), (2, 1, 0)):
        assert abs(O.csf_curvature(np.transpose(grid, perm).reshape(27)) - k0) < 1e-14
    for ax in range(3):
        assert abs(O.csf_curvature(np.flip(grid, ax).reshape(27)) - k0) < 1e-14


def test_csf_is_continuous_where_a_corner_gradient_vanishes():
    """Normals of corner gradients below 0.01 are shortened, not normalised:
    a liquid cell's stencil with one fill level changed by 1e-9 keeps a
    curvature of order 1e-7, and the curvature of a flat interface is
    unchanged by the floor."""
    phi = np.ones(27)
    assert O.csf_curvature(phi) == 0.0
    for i in range(27):
        p = phi.copy()
        p[i] -= 1e-9
        assert abs(O.csf_curvature(p)) < 1e-6
    flat = stencil(lambda x: np.clip(0.5 - 0.5 * x[2], 0, 1))
    assert abs(O.csf_curvature(flat)) < 1e-15
