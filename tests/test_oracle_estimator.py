"""Pins of the oracle's learned estimator as a lattice uses it (reading O18:
the network output corrects the finite-difference estimate of the same
fill stencil, with a per-cell fallback to finite differences).

* zero weights give the finite-difference estimate, on any stencil (the
  curvature exactly, the normal to the rounding of its renormalisation);
* bias-only networks on a planar stencil (whose finite-difference normal is
  exactly (0, 0, 1) and curvature exactly 0, pinned in the geometry tests)
  put the corrected normal and curvature on either side of each fallback
  threshold -- |n_raw| in [0.5, 2], 30 degrees, |kappa| <= 0.5 -- where the
  outcome is a closed form;
* a solid neighbour always keeps finite differences, and it is the first
  rule; a vanishing gradient (no finite-difference normal) falls back by the
  angle rule;
* a single-path network checks the input centring phi - 1/2 and the
  quarter weight of the curvature output in closed form;
* in a lattice: zero weights reproduce the plain oracle (bit for bit but
  for the rounding of the renormalised normals), weights that force the
  curvature rule everywhere reproduce it bit for bit, and the rule field marks
  exactly the interface cells next to a solid or a wall (counted by the test
  from the cell types) when the network is otherwise accepted.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2301_10674_amd import inputs as I

NP = 6212
OFF_B3 = NP - 4


def plane_z(centre=0.5):
    """Stencil of a horizontal surface: liquid below, gas above."""
    phi = np.zeros(27)
    for i in range(27):
        cz = i // 9 - 1
        phi[i] = 1.0 if cz < 0 else (centre if cz == 0 else 0.0)
    return phi


def bias_net(b):
    p = np.zeros(NP)
    p[OFF_B3:] = b
    return p


def test_zero_weights_give_finite_differences():
    rng = np.random.default_rng(11)
    P = np.zeros(NP)
    for _ in range(200):
        phi = rng.uniform(0, 1, 27)
        n, k, rule, q = O.estimator_compose(P, phi)
        nf, kf = O.normal_curvature(phi)
        assert np.abs(n - nf).max() < 4e-16 and k == kf
        assert rule == (4 if abs(kf) > 0.5 else 0)
        assert abs(q[0] - 1.0) < 1e-15 and q[1] < 1e-6


@pytest.mark.parametrize("b,rule,n_exp,k_exp", [
    # tilt along x: accepted below 30 degrees, rejected above
    ((0.5, 0, 0, 0), 0, (0.5 / math.sqrt(1.25), 0, 1 / math.sqrt(1.25)), 0.0),
    ((0.55, 0, 0, 0), 0, (0.55 / math.sqrt(1.3025), 0, 1 / math.sqrt(1.3025)), 0.0),
    ((0.6, 0, 0, 0), 3, (0, 0, 1), 0.0),
    ((0, -0.9, 0, 0), 3, (0, 0, 1), 0.0),
    # length of n_raw inside [0.5, 2] only
    ((0, 0, 0.9, 0), 0, (0, 0, 1), 0.0),
    ((0, 0, 1.2, 0), 2, (0, 0, 1), 0.0),
    ((0, 0, -0.4, 0), 0, (0, 0, 1), 0.0),
    ((0, 0, -0.6, 0), 2, (0, 0, 1), 0.0),
    # curvature: y3 / 4 is added, |kappa| <= 0.5 accepted
    ((0, 0, 0, 1.6), 0, (0, 0, 1), 0.4),
    ((0, 0, 0, -1.9), 0, (0, 0, 1), -0.475),
    ((0, 0, 0, 2.4), 4, (0, 0, 1), 0.0),
    ((0, 0, 0, -2.4), 4, (0, 0, 1), 0.0),
    # the length rule comes before the angle rule, the angle before the curvature
    ((3.0, 0, 0, 3.0), 2, (0, 0, 1), 0.0),
    ((0.9, 0, 0, 3.0), 3, (0, 0, 1), 0.0),
])
def test_bias_network_on_a_plane(b, rule, n_exp, k_exp):
    n, k, r, q = O.estimator_compose(bias_net(b), plane_z())
    assert r == rule
    assert np.allclose(n, n_exp, atol=1e-15, rtol=0) and abs(k - k_exp) < 1e-15
    nr = np.array([0, 0, 1.0]) + np.array(b[:3])
    assert abs(q[0] - np.linalg.norm(nr)) < 1e-15
    assert abs(q[1] - math.degrees(math.atan2(np.hypot(nr[0], nr[1]), nr[2]))) < 1e-9


def test_solid_neighbour_is_the_first_rule():
    for b in [(0, 0, 0, 0), (0.5, 0, 0, 0), (0, 0, 1.2, 0), (0.9, 0, 0, 3.0)]:
        n, k, r, _ = O.estimator_compose(bias_net(b), plane_z(), solid_nb=True)
        assert r == 1 and np.array_equal(n, [0, 0, 1.0]) and k == 0.0


def test_vanishing_gradient_falls_back_by_angle():
    phi = np.full(27, 0.5)
    n, k, r, q = O.estimator_compose(bias_net((1.0, 0, 0, 0)), phi)
    assert r == 3 and np.array_equal(n, np.zeros(3)) and k == 0.0 and abs(q[1] - 90.0) < 1e-12


def test_single_path_network_centres_the_input():
    """W1[0][rest] = 1, W2[0][0] = 1, W3[3][0] = 4 s: kappa = kappa_fd +
    s tanh(tanh(phi_c - 1/2)); the plane's kappa_fd is 0 for any centre
    fill, and the normal is untouched."""
    s = 0.3
    P = np.zeros(NP)
    P[0 * 27 + 13] = 1.0                      # W1[0][13]
    off_w2 = 64 * 27 + 64
    P[off_w2 + 0] = 1.0                       # W2[0][0]
    off_w3 = off_w2 + 64 * 64 + 64
    P[off_w3 + 3 * 64 + 0] = 4.0 * s          # W3[3][0]
    for c in (0.2, 0.5, 0.8):
        n, k, r, _ = O.estimator_compose(P, plane_z(c))
        assert r == 0 and np.array_equal(n, [0, 0, 1.0])
        assert abs(k - s * math.tanh(math.tanh(c - 0.5))) < 1e-15


def lattice_pair(w):
    def make():
        o = O.OracleLattice(w.shape, w.omega, accel=w.accel, sigma=w.sigma, fill=w.fill,
                            rho=w.rho, vel=w.vel)
        o.set_particles(w.centre, w.radius, w.sphere_vel, w.sphere_angvel)
        return o
    return make(), make()


def surface_spheres():
    return I.film_with_surface_spheres()


def solid_or_wall_neighbour(t):
    """Per cell: some 26-neighbour is solid or lies beyond a z wall."""
    nz = t.shape[0]
    out = np.zeros(t.shape, dtype=bool)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if dx == dy == dz == 0:
                    continue
                s = np.roll(t, (-dy, -dx), axis=(1, 2))
                nb = np.full(t.shape, O.SOLID, dtype=t.dtype)
                if dz == 0:
                    nb = s
                elif dz == 1:
                    nb[:nz - 1] = s[1:]
                else:
                    nb[1:] = s[:nz - 1]
                out |= nb == O.SOLID
    return out


def test_lattice_zero_weights_reproduce_the_plain_oracle():
    w = surface_spheres()
    a, b = lattice_pair(w)
    b.set_estimator(np.zeros(NP))
    for _ in range(3):
        a.step(4)
        b.step(4)
        for f in (O.F_TYPE, O.F_MASS, O.F_PDF, O.F_CURV):
            assert np.array_equal(a.read(f), b.read(f)), f
        assert np.abs(a.read(O.F_NORMAL) - b.read(O.F_NORMAL)).max() < 4e-16
    t = b.read(O.F_TYPE)
    rule = b.read(O.F_EST_RULE)
    itf = t == O.INTERFACE
    near = solid_or_wall_neighbour(t) & itf
    assert near.sum() > 20 and (itf & ~near).sum() > 100
    assert np.all(rule[near] == O.EST_SOLID)
    # finite differences agree with themselves to the angle rule's rounding
    assert np.all(np.isin(rule[itf & ~near], [O.EST_NETWORK, O.EST_KAPPA]))
    assert np.all(rule[~itf] == 0)


def test_lattice_rejected_corrections_change_nothing():
    w = surface_spheres()
    a, b = lattice_pair(w)
    b.set_estimator(bias_net((0.3, -0.2, 0.1, 100.0)))   # |kappa| > 0.5 everywhere
    a.step(6)
    b.step(6)
    for f in (O.F_TYPE, O.F_MASS, O.F_PDF, O.F_NORMAL, O.F_CURV):
        assert np.array_equal(a.read(f), b.read(f)), f
    t = b.read(O.F_TYPE)
    itf = t == O.INTERFACE
    near = solid_or_wall_neighbour(t) & itf
    rule = b.read(O.F_EST_RULE)
    assert np.all(rule[near] == O.EST_SOLID) and np.all(rule[itf & ~near] == O.EST_KAPPA)


def test_lattice_accepted_corrections_are_used():
    """A bias that tilts every normal by 14 degrees towards +x is accepted
    away from solids and moves the stored normals; mass stays exact."""
    w = surface_spheres()
    _, b = lattice_pair(w)
    M0 = b.total_mass()
    nf0 = b.read(O.F_NORMAL).copy()
    b.set_estimator(bias_net((0.25, 0.0, 0.0, 0.0)))
    t = b.read(O.F_TYPE)
    itf = t == O.INTERFACE
    near = solid_or_wall_neighbour(t) & itf
    rule = b.read(O.F_EST_RULE)
    far = itf & ~near
    acc = far & (rule == O.EST_NETWORK)
    assert acc.sum() > 0.9 * far.sum()
    n = b.read(O.F_NORMAL)
    raw = nf0[:, acc] + np.array([0.25, 0, 0])[:, None]
    assert np.allclose(n[:, acc], raw / np.linalg.norm(raw, axis=0), atol=1e-14, rtol=0)
    assert np.array_equal(n[:, near], nf0[:, near])
    b.step(10)
    assert abs(b.total_mass() - M0) < 1e-12 * M0
