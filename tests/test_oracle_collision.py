"""Pins of the oracle's lattice tables and cumulant collision.

The oracle follows Geier et al. (2015) as Section 2.1 prescribes it: chimera
passes, cumulant relations, relaxation with omega for shear and 1 for every
other rate.  These tests check it against things that do not share its
shortcuts:

* the D3Q27 weight identities (Section 2.1, D3Q27 lattice);
* a brute-force collision: central moments by direct sums, cumulants by the
  set-partition (Moebius) formula, relaxation written as deviator + trace,
  moments rebuilt by the partition sum, PDFs by solving the 27 x 27 moment
  system -- for arbitrary rates, so every cumulant order is exercised;
* closed forms: all rates 1 and no force give the product-form equilibrium,
  the equilibrium is a fixed point, the identity for all rates 0;
* conservation of mass and of momentum plus force;
* equivariance under the 48 symmetries of the cube.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import oracle as O

C, W = O.velocities()


def test_weights_and_isotropy():
    assert abs(W.sum() - 1.0) < 1e-15
    for i in range(27):
        assert tuple(C[26 - i]) == tuple(-C[i])
        assert W[26 - i] == W[i]
    assert tuple(C[13]) == (0, 0, 0)
    assert abs(W[13] - 8.0 / 27.0) < 1e-16
    for a in range(3):
        assert abs((W * C[:, a]).sum()) < 1e-16
        for b in range(3):
            m2 = (W * C[:, a] * C[:, b]).sum()
            assert abs(m2 - (1.0 / 3.0 if a == b else 0.0)) < 1e-15
            m4 = (W * C[:, a] ** 2 * C[:, b] ** 2).sum()
            assert abs(m4 - (1.0 / 3.0 if a == b else 1.0 / 9.0)) < 1e-15
    assert abs((W * (C[:, 0] * C[:, 1] * C[:, 2]) ** 2).sum() - 1.0 / 27.0) < 1e-15


# ---------------------------------------------------------------- brute force
def set_partitions(items):
    if not items:
        yield []
        return
    first, rest = items[0], items[1:]
    for part in set_partitions(rest):
        for k in range(len(part)):
            yield part[:k] + [[first] + part[k]] + part[k + 1:]
        yield [[first]] + part


def labels(idx):
    a, b, c = idx
    return [0] * a + [1] * b + [2] * c


def block_index(block):
    return (block.count(0), block.count(1), block.count(2))


MULTI = [(a, b, c) for c in range(3) for b in range(3) for a in range(3)]  # i = a+3b+9c


def brute_central(f, u):
    rho = f.sum()
    k = {}
    for idx in MULTI:
        a, b, c = idx
        k[idx] = float((f * (C[:, 0] - u[0]) ** a * (C[:, 1] - u[1]) ** b
                        * (C[:, 2] - u[2]) ** c).sum() / rho)
    return rho, k


def brute_cumulant(idx, k):
    """Cumulant of the multiset idx from normalised central moments k, with
    the first-order moments taken as zero (blocks of size 1 vanish)."""
    tot = 0.0
    for part in set_partitions(labels(idx)):
        if any(len(B) == 1 for B in part):
            continue
        nb = len(part)
        term = (-1) ** (nb - 1) * math.factorial(nb - 1)
        for B in part:
            term *= k[block_index(B)]
        tot += term
    return tot


def brute_moment(idx, cum):
    tot = 0.0
    for part in set_partitions(labels(idx)):
        if any(len(B) == 1 for B in part):
            continue
        term = 1.0
        for B in part:
            term *= cum[block_index(B)]
        tot += term
    return tot


def brute_collide(f, g, omega, omega_bulk, omega_high):
    rho = f.sum()
    j = (f[:, None] * C).sum(axis=0)
    u = (j + 0.5 * rho * np.asarray(g)) / rho
    rho, k = brute_central(f, u)
    cum = {idx: brute_cumulant(idx, k) for idx in MULTI if sum(idx) >= 2}
    # second order: deviator with omega, trace with omega_bulk towards 1
    Kt = np.zeros((3, 3))
    for a in range(3):
        for b in range(3):
            e = [0, 0, 0]
            e[a] += 1
            e[b] += 1
            Kt[a, b] = cum[tuple(e)]
    tr = np.trace(Kt)
    Ks = (1 - omega) * (Kt - tr / 3 * np.eye(3)) + ((1 - omega_bulk) * tr + omega_bulk) / 3 * np.eye(3)
    cs = {}
    for idx in cum:
        if sum(idx) == 2:
            ab = [d for d in range(3) for _ in range(idx[d])]
            cs[idx] = Ks[ab[0], ab[1]]
        else:
            cs[idx] = (1 - omega_high) * cum[idx]
    ks = {idx: brute_moment(idx, cs) for idx in cs}
    ks[(0, 0, 0)] = 1.0
    for d in range(3):
        e = [0, 0, 0]
        e[d] = 1
        ks[tuple(e)] = -k[tuple(e)]
    # solve sum_i f_i prod (c - u)^alpha = rho k*_alpha
    V = np.zeros((27, 27))
    rhs = np.zeros(27)
    for r, idx in enumerate(MULTI):
        a, b, c = idx
        V[r] = (C[:, 0] - u[0]) ** a * (C[:, 1] - u[1]) ** b * (C[:, 2] - u[2]) ** c
        rhs[r] = rho * ks[idx]
    return np.linalg.solve(V, rhs), cum


def random_state(rng, amp=0.05):
    rho = 1.0 + 0.02 * rng.standard_normal()
    u = 0.05 * rng.standard_normal(3)
    f = O.feq(rho, u) * (1.0 + amp * rng.standard_normal(27))
    return f


@pytest.mark.parametrize("seed", range(6))
def test_collision_matches_brute_force(seed):
    rng = np.random.default_rng(seed)
    f = random_state(rng)
    g = 1e-3 * rng.standard_normal(3)
    omega = rng.uniform(0.2, 1.99)
    ob = rng.uniform(0.3, 1.7) if seed % 2 else 1.0
    oh = rng.uniform(0.3, 1.7) if seed % 2 else 1.0
    fo = O.collide(f, g, omega, ob, oh)
    fb, cum = brute_collide(f, g, omega, ob, oh)
    assert np.max(np.abs(fo - fb)) < 1e-13
    # the oracle's own cumulants, order >= 2
    co = O.cumulants(f, g)
    for i, idx in enumerate(MULTI):
        if sum(idx) >= 2:
            assert abs(co[i] - cum[idx]) < 1e-14, idx


def test_all_rates_zero_is_identity():
    rng = np.random.default_rng(5)
    for _ in range(5):
        f = random_state(rng, amp=0.2)
        fo = O.collide(f, (0, 0, 0), 0.0, 0.0, 0.0)
        assert np.max(np.abs(fo - f)) < 1e-15


def product_equilibrium(rho, u):
    out = np.zeros(27)
    for i in range(27):
        p = rho
        for d in range(3):
            c = C[i, d]
            p *= (2.0 / 3.0 - u[d] ** 2) if c == 0 else 0.5 * (1.0 / 3.0 + u[d] ** 2 + c * u[d])
        out[i] = p
    return out


def test_unit_rates_give_product_equilibrium():
    rng = np.random.default_rng(7)
    for _ in range(10):
        f = random_state(rng, amp=0.3)
        rho = f.sum()
        u = (f[:, None] * C).sum(0) / rho
        fo = O.collide(f, (0, 0, 0), 1.0, 1.0, 1.0)
        assert np.max(np.abs(fo - product_equilibrium(rho, u))) < 1e-15


def test_equilibrium_is_fixed_point():
    rng = np.random.default_rng(8)
    for omega in (0.5, 1.0, 1.5, 1.9, 1.997):
        rho = 1.0 + 0.05 * rng.standard_normal()
        u = 0.08 * rng.standard_normal(3)
        fe = O.feq(rho, u)
        assert np.max(np.abs(fe - product_equilibrium(rho, u))) < 1e-16
        fo = O.collide(fe, (0, 0, 0), omega)
        assert np.max(np.abs(fo - fe)) < 1e-15


def test_mass_and_momentum_with_force():
    rng = np.random.default_rng(9)
    for _ in range(10):
        f = random_state(rng, amp=0.3)
        g = 1e-3 * rng.standard_normal(3)
        fo = O.collide(f, g, rng.uniform(0.5, 1.99))
        rho = f.sum()
        assert abs(fo.sum() - rho) < 1e-15
        j = (f[:, None] * C).sum(0)
        jo = (fo[:, None] * C).sum(0)
        assert np.max(np.abs(jo - (j + rho * g))) < 1e-15


def cube_symmetries():
    mats = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            R = np.zeros((3, 3), dtype=int)
            for r in range(3):
                R[r, perm[r]] = signs[r]
            mats.append(R)
    return mats


def test_cube_symmetry_equivariance():
    rng = np.random.default_rng(10)
    f = random_state(rng, amp=0.2)
    g = 1e-3 * rng.standard_normal(3)
    fo = O.collide(f, g, 1.7)
    index = {tuple(C[i]): i for i in range(27)}
    syms = cube_symmetries()
    assert len(syms) == 48
    for R in syms:
        perm = np.array([index[tuple(R @ C[i])] for i in range(27)])
        fr = np.zeros(27)
        fr[perm] = f
        for_ = np.zeros(27)
        for_[perm] = fo
        got = O.collide(fr, R @ g, 1.7)
        assert np.max(np.abs(got - for_)) < 1e-15
