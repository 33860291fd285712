"""Seeded synthetic inputs for the free-surface lattice.

This module only builds initial conditions (fill level, density, velocity,
spheres and physical parameters).  It holds none of the method's arithmetic,
so both the GPU path and the CPU oracle can consume its output.

Workloads (all lattice units):

* ``channel_film``: the parity configuration -- 64 x 8 x 32, periodic x/y,
  walls at both z ends, liquid up to z = 20 + 2 sin(2 pi x / 64), 16 fixed
  spheres of radius 3 in z < 8, body force g_x = 1e-5, omega = 1.9.
* ``flume``: a sediment flume shaped like the paper's setup (Section 3.1):
  a bed of three layers of diameter-10 spheres (a jittered hexagonal base
  layer plus two jittered close-packed layers), a flat free surface 60 cells
  above the bed, hydrostatic density, a parabolic velocity profile above the
  bed with 1 % noise, gravity from Fr = 1.3, slope tan(psi) = 0.044 (Table 2,
  run E1), omega = 1.997 and sigma from We = 15.62 (Table 1, run E1).
  Fluid pockets that the spheres enclose completely start as gas: the
  spheres move by prescribed velocities that their cells do not follow, so
  moving bounce-back on the walls of a closed pocket between spheres of
  different velocities adds or removes mass there every step, without
  bound.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Workload:
    name: str
    shape: tuple                   # (nx, ny, nz)
    omega: float
    accel: tuple                   # body acceleration (gx, gy, gz)
    sigma: float
    fill: np.ndarray               # (nz, ny, nx)
    rho: np.ndarray                # (nz, ny, nx)
    vel: np.ndarray                # (3, nz, ny, nx)
    centre: np.ndarray             # (n, 3)
    radius: np.ndarray             # (n,)
    sphere_vel: np.ndarray         # (n, 3)
    sphere_angvel: np.ndarray      # (n, 3)
    rho_gas: float = 1.0
    conv_eps: float = 1e-2
    meta: dict = field(default_factory=dict)

    @property
    def ncells(self):
        nx, ny, nz = self.shape
        return nx * ny * nz


def height_fill(shape, h):
    """Fill level of cells below a height field h[y, x]: cell k holds the
    fraction of [k, k+1] that lies under the surface."""
    nx, ny, nz = shape
    k = np.arange(nz, dtype=np.float64)[:, None, None]
    return np.clip(np.asarray(h, dtype=np.float64)[None, :, :] - k, 0.0, 1.0)


def channel_film(seed: int = 1) -> Workload:
    nx, ny, nz = 64, 8, 32
    rng = np.random.Generator(np.random.PCG64(seed))
    xc = np.arange(nx) + 0.5
    h = 20.0 + 2.0 * np.sin(2.0 * np.pi * xc / nx)
    fill = height_fill((nx, ny, nz), np.broadcast_to(h[None, :], (ny, nx)))
    n = 16
    centre = np.stack([rng.uniform(0.0, nx, n), rng.uniform(0.0, ny, n),
                       rng.uniform(3.0, 8.0, n)], axis=1)
    radius = np.full(n, 3.0)
    return Workload(
        name="channel_film_64x8x32", shape=(nx, ny, nz), omega=1.9,
        accel=(1e-5, 0.0, 0.0), sigma=0.0, fill=fill,
        rho=np.ones((nz, ny, nx)), vel=np.zeros((3, nz, ny, nx)),
        centre=centre, radius=radius, sphere_vel=np.zeros((n, 3)),
        sphere_angvel=np.zeros((n, 3)),
        meta={"seed": seed, "steps": 200})


def film_with_surface_spheres(sigma: float = 0.0, nz: int = 32) -> Workload:
    """The channel film with four more fixed spheres of radius 3 centred on
    its free surface (x = 8, 24, 40, 56; y = 4), so that interface cells
    touch solids; with nz = 22 the surface crests (z up to 22) also reach
    the top wall."""
    w = channel_film()
    nx, ny, _ = w.shape
    xs = np.array([8.0, 24.0, 40.0, 56.0])
    h = 20.0 + 2.0 * np.sin(2.0 * np.pi * xs / nx)
    extra = np.stack([xs, np.full(4, 4.0), h], axis=1)
    n = len(w.radius) + 4
    xc = np.arange(nx) + 0.5
    hh = 20.0 + 2.0 * np.sin(2.0 * np.pi * xc / nx)
    fill = height_fill((nx, ny, nz), np.broadcast_to(hh[None, :], (ny, nx)))
    return Workload(
        name="film_surface_spheres_%dx%dx%d" % (nx, ny, nz), shape=(nx, ny, nz), omega=w.omega,
        accel=w.accel, sigma=sigma, fill=fill, rho=np.ones((nz, ny, nx)),
        vel=np.zeros((3, nz, ny, nx)), centre=np.concatenate([w.centre, extra]),
        radius=np.concatenate([w.radius, np.full(4, 3.0)]), sphere_vel=np.zeros((n, 3)),
        sphere_angvel=np.zeros((n, 3)), meta={"seed": 1})


def _bed_spheres(nx, ny, rng, d=10.0, layers=3, z0=5.0, jitter=0.75):
    """Jittered hexagonal packing of ``layers`` layers of diameter-d spheres
    that tiles the periodic nx x ny box."""
    ncol = max(1, int(round(nx / d)))
    nrow = max(2, 2 * int(round(ny / (d * math.sqrt(3.0)))))
    sx, sy = nx / ncol, ny / nrow
    dz = d * math.sqrt(2.0 / 3.0)
    out = []
    for layer in range(layers):
        zl = z0 + layer * dz
        ox = (layer % 3) * sx / 3.0
        oy = (layer % 3) * sy / 3.0
        for r in range(nrow):
            for c in range(ncol):
                x = (c + 0.5 * (r % 2)) * sx + ox
                y = (r + 0.5) * sy + oy
                out.append((x, y, zl))
    p = np.array(out, dtype=np.float64)
    p[:, 0] += rng.uniform(-jitter, jitter, len(p))
    p[:, 1] += rng.uniform(-jitter, jitter, len(p))
    p[:, 2] += rng.uniform(-0.5 * jitter, 0.5 * jitter, len(p))
    p[:, 0] %= nx
    p[:, 1] %= ny
    return p


def _solid_fraction_profile(shape, centre, radius):
    """y-averaged solid fraction per (z, x) of the sphere bed (cell centres)."""
    nx, ny, nz = shape
    solid = np.zeros((nz, ny, nx), dtype=bool)
    zc = np.arange(nz) + 0.5
    yc = np.arange(ny) + 0.5
    xc = np.arange(nx) + 0.5
    for (X, Y, Z), r in zip(centre, radius):
        z0, z1 = max(0, int(Z - r) - 1), min(nz, int(Z + r) + 2)
        dz = zc[z0:z1, None, None] - Z
        dy = yc[None, :, None] - Y
        dy = dy - ny * np.round(dy / ny)
        x0, x1 = int(math.floor(X - r)) - 1, int(math.floor(X + r)) + 2
        xi = np.arange(x0, x1) % nx
        dx = xc[xi][None, None, :] - X
        dx = dx - nx * np.round(dx / nx)
        inside = dx * dx + dy * dy + dz * dz <= r * r
        solid[z0:z1, :, xi] |= inside
    return solid.mean(axis=1)  # (nz, nx)


def bed_height(shape, centre, radius, level=0.3):
    """Bed height where the y-averaged solid fraction drops to ``level``
    (Section 3.2: linear interpolation of phi_b(x, z) = 0.3), averaged in x."""
    phib = _solid_fraction_profile(shape, centre, radius)
    nz = phib.shape[0]
    hs = []
    for col in phib.T:
        k = nz - 1
        while k > 0 and col[k] < level:
            k -= 1
        if k >= nz - 1 or col[k] < level:
            hs.append(0.0)
            continue
        # col[k] >= level > col[k+1]: interpolate between cell centres
        t = (col[k] - level) / (col[k] - col[k + 1])
        hs.append(k + 0.5 + t)
    return float(np.mean(hs))


def _solid_cells(shape, centre, radius, shrink=1e-9):
    """Cells whose centre lies within radius - shrink of a sphere centre
    (periodic in x and y): a subset of the cells the lattice makes solid."""
    nx, ny, nz = shape
    solid = np.zeros((nz, ny, nx), dtype=bool)
    zc, yc, xc = (np.arange(n) + 0.5 for n in (nz, ny, nx))
    for (X, Y, Z), r in zip(centre, radius):
        r = r - shrink
        z0, z1 = max(0, int(math.floor(Z - r)) - 1), min(nz, int(math.floor(Z + r)) + 2)
        yi = np.arange(int(math.floor(Y - r)) - 1, int(math.floor(Y + r)) + 2) % ny
        xi = np.arange(int(math.floor(X - r)) - 1, int(math.floor(X + r)) + 2) % nx
        dz = zc[z0:z1, None, None] - Z
        dy = yc[yi][None, :, None] - Y
        dy = dy - ny * np.round(dy / ny)
        dx = xc[xi][None, None, :] - X
        dx = dx - nx * np.round(dx / nx)
        inside = dx * dx + dy * dy + dz * dz <= r * r
        blk = solid[z0:z1][:, yi][:, :, xi] | inside
        solid[np.ix_(np.arange(z0, z1), yi, xi)] = blk
    return solid


def enclosed_pockets(fill, solid):
    """Fluid cells (fill > 0, not solid) that no chain of D3Q27 links
    between fluid cells joins to the free surface (a fluid cell with fill
    below 1 or with a gas neighbour); the box is periodic in x and y and
    closed in z.  ``solid`` may miss cells at sphere surfaces: extra fluid
    cells can only join pockets to the surface, so every cell returned is
    enclosed."""
    from scipy import ndimage
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components

    fluid = (fill > 0.0) & ~solid
    ball = np.ones((3, 3, 3), dtype=bool)
    lab, n = ndimage.label(fluid, structure=ball)
    if n == 0:
        return np.zeros_like(fluid)
    # links across the periodic x and y faces (the roll along the face's
    # other axis wraps too, which covers the links across both at once)
    a, b = [], []
    for axis in (2, 1):
        lo = np.take(lab, 0, axis=axis)
        hi = np.take(lab, -1, axis=axis)
        for dz in (-1, 0, 1):
            for dt in (-1, 0, 1):
                h = np.roll(hi, dt, axis=1)
                l2 = lo
                if dz > 0:
                    h, l2 = h[dz:], lo[:-dz]
                elif dz < 0:
                    h, l2 = h[:dz], lo[-dz:]
                m = (h > 0) & (l2 > 0)
                a.append(h[m])
                b.append(l2[m])
    a, b = np.concatenate(a), np.concatenate(b)
    g = coo_matrix((np.ones(len(a)), (a, b)), shape=(n + 1, n + 1))
    _, comp = connected_components(g, directed=False)
    gas = (fill <= 0.0) & ~solid
    near_gas = ndimage.binary_dilation(np.pad(gas, ((0, 0), (1, 1), (1, 1)), mode="wrap"),
                                       structure=ball)[:, 1:-1, 1:-1]
    surface = fluid & ((fill < 1.0) | near_gas)
    if not surface.any():
        return np.zeros_like(fluid)
    keep = np.zeros(n + 1, dtype=bool)
    keep[np.unique(comp[lab[surface]])] = True
    return fluid & ~keep[comp[lab]]


def flume(nx: int = 1536, ny: int = 40, nz: int = 192, seed: int = 2,
          depth: float = 60.0, U: float = 0.02, Fr: float = 1.3,
          We: float = 15.62, slope: float = 0.044, omega: float = 1.997,
          noise: float = 0.01, d: float = 10.0, layers: int = 3,
          sphere_speed: float = 1e-4) -> Workload:
    rng = np.random.Generator(np.random.PCG64(seed))
    centre = _bed_spheres(nx, ny, rng, d=d, layers=layers)
    n = len(centre)
    radius = np.full(n, 0.5 * d)
    hb = bed_height((nx, ny, nz), centre, radius)
    zs = hb + depth
    if zs >= nz - 2:
        raise ValueError("free surface does not fit below the top wall")
    g = (U / Fr) ** 2 / depth            # Fr = U / sqrt(g h0)
    gx = slope * g                       # depth-slope driving, tan(psi)
    sigma = U * U * depth / We           # We = rho U^2 h0 / sigma
    fill = height_fill((nx, ny, nz), np.full((ny, nx), zs))
    pockets = enclosed_pockets(fill, _solid_cells((nx, ny, nz), centre, radius))
    fill[pockets] = 0.0
    zc = (np.arange(nz) + 0.5)[:, None, None]
    rho = np.exp(3.0 * g * np.clip(zs - zc, 0.0, None)) * np.ones((1, ny, nx))
    zeta = np.clip((zc - hb) / depth, 0.0, 1.0)
    ux = 1.5 * U * (2.0 * zeta - zeta * zeta) * np.ones((1, ny, nx))
    vel = np.zeros((3, nz, ny, nx))
    vel[0] = ux
    liquid = fill > 0.0
    vel += noise * U * rng.standard_normal((3, nz, ny, nx)) * liquid[None]
    svel = rng.uniform(-sphere_speed, sphere_speed, (n, 3))
    return Workload(
        name=f"flume_{nx}x{ny}x{nz}", shape=(nx, ny, nz), omega=omega,
        accel=(gx, 0.0, -g), sigma=sigma, fill=fill, rho=rho, vel=vel,
        centre=centre, radius=radius, sphere_vel=svel,
        sphere_angvel=np.zeros((n, 3)),
        meta={"seed": seed, "bed_height": hb, "surface": zs, "spheres": n,
              "enclosed_cells": int(pockets.sum()),
              "depth": depth, "U": U, "Fr": Fr, "We": We, "slope": slope})


def flume_crop(nx: int = 128, seed: int = 3, **kw) -> Workload:
    """The flume recipe on its own short periodic box (accuracy crop)."""
    return flume(nx=nx, seed=seed, **kw)


def flat_film(shape=(4, 4, 24), h=16.5, omega=1.0, gx=1e-6, gz=0.0, sigma=0.0):
    """Flat liquid film of height h on the bottom wall, at rest."""
    nx, ny, nz = shape
    fill = height_fill(shape, np.full((ny, nx), h))
    return Workload(
        name="flat_film", shape=shape, omega=omega, accel=(gx, 0.0, gz),
        sigma=sigma, fill=fill, rho=np.ones((nz, ny, nx)),
        vel=np.zeros((3, nz, ny, nx)), centre=np.zeros((0, 3)),
        radius=np.zeros(0), sphere_vel=np.zeros((0, 3)),
        sphere_angvel=np.zeros((0, 3)), meta={"h": h})


def droplet(n: int = 40, radius: float = 10.0, sigma: float = 1e-3, omega: float = 1.0,
            ss: int = 4) -> Workload:
    """Static droplet of the given radius centred in an n^3 box at rest, no
    gravity; fill levels by supersampling each cell on an ss^3 grid."""
    o = (np.arange(ss) + 0.5) / ss
    g = np.arange(n) - 0.5 * n
    fill = np.zeros((n, n, n))
    for a in o:
        for b in o:
            for c in o:
                z = (g + a)[:, None, None]
                y = (g + b)[None, :, None]
                x = (g + c)[None, None, :]
                fill += x * x + y * y + z * z <= radius * radius
    fill /= ss ** 3
    return Workload(
        name="droplet_%d_r%g" % (n, radius), shape=(n, n, n), omega=omega, accel=(0.0, 0.0, 0.0),
        sigma=sigma, fill=fill, rho=np.ones((n, n, n)), vel=np.zeros((3, n, n, n)),
        centre=np.zeros((0, 3)), radius=np.zeros(0), sphere_vel=np.zeros((0, 3)),
        sphere_angvel=np.zeros((0, 3)), meta={"radius": radius})


def splash(shape=(48, 32, 40), seed: int = 4, sigma: float = 1e-3) -> Workload:
    """A falling blob over a rough pool: liquid up to z = nz/3 with a noisy
    surface, a ball of radius nz/6 centred at 0.62 nz moving down at 0.04
    with a random swirl, gravity 2e-4 down.  The blob's edge and the pool's
    surface carry interface cells with only gas or only liquid neighbours,
    and the impact fills and empties many cells a step."""
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    h = nz / 3.0 + 0.8 * rng.standard_normal((ny, nx))
    fill = height_fill(shape, h)
    z, y, x = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5, np.arange(nx) + 0.5, indexing="ij")
    r = np.sqrt((x - 0.5 * nx) ** 2 + (y - 0.5 * ny) ** 2 + (z - 0.62 * nz) ** 2)
    ball = np.clip(nz / 6.0 + 0.5 - r, 0.0, 1.0)
    fill = np.clip(fill + ball, 0.0, 1.0)
    edge = (fill > 0) & (fill < 1)
    fill = np.where(edge, np.clip(fill + 0.15 * rng.standard_normal(fill.shape), 0.0, 1.0), fill)
    vel = np.zeros((3, nz, ny, nx))
    inball = r < nz / 6.0 + 1.0
    vel[2] = np.where(inball, -0.04, 0.0)
    vel += 0.01 * rng.standard_normal((3, nz, ny, nx)) * inball
    return Workload(name="splash_%dx%dx%d" % shape, shape=shape, omega=1.6, accel=(0.0, 0.0, -2e-4),
                    sigma=sigma, fill=fill, rho=np.ones((nz, ny, nx)), vel=vel,
                    centre=np.zeros((0, 3)), radius=np.zeros(0), sphere_vel=np.zeros((0, 3)),
                    sphere_angvel=np.zeros((0, 3)))


def sphere_cluster(box=(48, 36, 30), seed: int = 6):
    """60 spheres of radius 2.5-4 on a jittered 5 x 4 x 3 grid (spacing
    9.6 x 9 x 9, jitter +-1.2: close pairs that collide soon), with
    random velocities (0.03) and spins (0.002); the first six fixed."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = box
    g = np.stack(np.meshgrid((np.arange(5) + 0.5) * nx / 5, (np.arange(4) + 0.5) * ny / 4,
                             5.0 + 9.0 * np.arange(3), indexing="ij"), axis=-1).reshape(-1, 3)
    n = len(g)
    c = g + rng.uniform(-1.2, 1.2, (n, 3))
    r = rng.uniform(2.5, 4.0, n)
    v = 0.03 * rng.standard_normal((n, 3))
    w = 0.002 * rng.standard_normal((n, 3))
    fixed = np.zeros(n, dtype=np.uint8)
    fixed[: n // 10] = 1
    v[fixed == 1] = 0.0
    w[fixed == 1] = 0.0
    return c, r, v, w, fixed


def settling_box(shape=(24, 20, 28), seed: int = 8) -> Workload:
    """Liquid at rest to z = 20 under gravity 1e-3 down, three spheres of
    radius 3 moving down at 0.02 (one 0.3 cells above the bottom wall, one
    a few cells above it, one at the surface), for the coupled fluid-particle
    step."""
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    h = np.full((ny, nx), 20.0)
    fill = height_fill(shape, h)
    g = 1e-3
    z = np.arange(nz, dtype=np.float64)[:, None, None] + 0.5
    rho = np.exp(3.0 * g * (20.0 - np.minimum(z, 20.0))) * np.ones((nz, ny, nx))
    centre = np.array([[6.0, 5.0, 3.3], [15.5, 12.0, 9.0], [10.0, 15.0, 19.0]])
    centre[:, :2] += rng.uniform(-0.5, 0.5, (3, 2))
    return Workload(name="settling_%dx%dx%d" % shape, shape=shape, omega=1.5, accel=(0.0, 0.0, -g),
                    sigma=0.0, fill=fill, rho=rho, vel=np.zeros((3, nz, ny, nx)), centre=centre,
                    radius=np.full(3, 3.0), sphere_vel=np.tile([0.0, 0.0, -0.02], (3, 1)),
                    sphere_angvel=np.zeros((3, 3)))
