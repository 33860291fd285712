"""The flume recipe's enclosed-pocket search against a brute-force flood
fill over D3Q27 links (periodic x and y, closed z) on tiny boxes: hand-built
cases (a closed cavity; regions joined to the surface only across the
periodic x or y face, or across both at once) and random solids."""
from collections import deque

import numpy as np
import pytest

from paper_2301_10674_amd import inputs as I


def brute_force(fill, solid):
    nz, ny, nx = fill.shape
    fluid = (fill > 0) & ~solid
    gas = (fill <= 0) & ~solid
    reach = np.zeros_like(fluid)
    q = deque()

    def nbrs(z, y, x):
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    if (dz or dy or dx) and 0 <= z + dz < nz:
                        yield z + dz, (y + dy) % ny, (x + dx) % nx

    for z, y, x in zip(*np.nonzero(fluid)):
        if fill[z, y, x] < 1 or any(gas[c] for c in nbrs(z, y, x)):
            reach[z, y, x] = True
            q.append((z, y, x))
    if not q:
        return np.zeros_like(fluid)
    while q:
        for c in nbrs(*q.popleft()):
            if fluid[c] and not reach[c]:
                reach[c] = True
                q.append(c)
    return fluid & ~reach


def layer_fill(shape, h):
    nz, ny, nx = shape
    return np.clip(h - np.arange(nz, dtype=float), 0.0, 1.0)[:, None, None] * np.ones((1, ny, nx))


def test_closed_cavity():
    fill = layer_fill((10, 8, 8), 7.5)
    solid = np.zeros(fill.shape, bool)
    solid[1:6, 1:6, 1:6] = True
    solid[2:5, 2:5, 2:5] = False          # a 3x3x3 cavity inside a closed shell
    got = I.enclosed_pockets(fill, solid)
    assert got.sum() == 27 and got[2:5, 2:5, 2:5].all()
    assert np.array_equal(got, brute_force(fill, solid))


@pytest.mark.parametrize("axis", ["x", "y", "xy"])
def test_region_joined_across_periodic_faces(axis):
    """Cells under a roof whose only way to the surface crosses the
    periodic face(s): they are not enclosed."""
    nz, ny, nx = 8, 6, 6
    fill = layer_fill((nz, ny, nx), 6.5)
    solid = np.zeros((nz, ny, nx), bool)
    solid[3] = True                       # a roof over z < 3 ...
    if axis == "x":
        solid[3, :, nx - 1] = False       # ... open above the column x = nx-1
        solid[:3, :, nx - 2] = True       # ... walled off from it inside the box
    elif axis == "y":
        solid[3, ny - 1, :] = False
        solid[:3, ny - 2, :] = True
    else:
        solid[3, ny - 1, nx - 1] = False  # one open column at the far corner
        solid[:3, ny - 2, :] = True       # walls on both sides inside the box
        solid[:3, :, nx - 2] = True
    got = I.enclosed_pockets(fill, solid)
    assert np.array_equal(got, brute_force(fill, solid))
    assert not got.any()
    # closing the opening makes the region under the roof a pocket
    solid[3] = True
    got = I.enclosed_pockets(fill, solid)
    assert np.array_equal(got, brute_force(fill, solid))
    assert got[:3].sum() == ((~solid[:3]).sum())


def random_case(seed):
    """A shell of solid cells at a random place (it may straddle the
    periodic faces), with a hole in half of the cases, random solids inside
    and outside it, liquid up to a random level above it."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = 10, int(rng.integers(6, 9)), int(rng.integers(6, 9))
    fill = layer_fill((nz, ny, nx), 7.0 + rng.uniform(0.1, 0.9))
    solid = rng.random((nz, ny, nx)) < 0.25
    z0, y0, x0 = int(rng.integers(0, 3)), int(rng.integers(0, ny)), int(rng.integers(0, nx))
    a = int(rng.integers(4, 6))
    zs = np.arange(z0, z0 + a)
    ys, xs = (y0 + np.arange(a)) % ny, (x0 + np.arange(a)) % nx
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    edge = (Z == zs[0]) | (Z == zs[-1]) | (Y == ys[0]) | (Y == ys[-1]) | (X == xs[0]) | (X == xs[-1])
    solid[Z[edge], Y[edge], X[edge]] = True
    solid[Z[~edge], Y[~edge], X[~edge]] = rng.random(int((~edge).sum())) < 0.3
    if rng.random() < 0.5:
        k = rng.integers(0, int(edge.sum()))
        solid[Z[edge][k], Y[edge][k], X[edge][k]] = False
    solid[z0 + a:][fill[z0 + a:] < 1.0] = False
    return fill, solid


def test_random_shells():
    found = 0
    for seed in range(40):
        fill, solid = random_case(seed)
        want = brute_force(fill, solid)
        assert np.array_equal(I.enclosed_pockets(fill, solid), want), seed
        found += bool(want.any())
    assert 10 <= found <= 35, found      # both kinds of case occur


def test_flume_pockets_start_as_gas():
    """In the generated flume no fluid cell is enclosed."""
    w = I.flume(nx=64, ny=80, nz=128, seed=11, depth=30.0)
    solid = I._solid_cells(w.shape, w.centre, w.radius)
    assert not I.enclosed_pockets(w.fill, solid).any()
    assert w.meta["enclosed_cells"] >= 0
