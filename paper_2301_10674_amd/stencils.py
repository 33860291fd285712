"""Training and test stencils for the learned interface estimator.

A sample is the 3x3x3 fill-level stencil around an interface cell (entry
k = a + 3b + 9c holds the cell at offset (a-1, b-1, c-1)) and a label: the
unit normal pointing from liquid to gas and the mean curvature kappa
(positive for convex liquid, so that 2 sigma kappa is the Laplace pressure
of Section 2.1).

* ``analytic_stencils``: seeded droplets / bubbles (radius log-uniform in
  [4, 64]) and sinusoidal sheets (minimum radius of curvature log-uniform in
  [4, 64], random orientation and phase); fill levels by supersampling each
  cell on an ss^3 grid; labels exact at the surface point nearest to the
  centre of the stencil.
* ``height_function_samples``: interface cells of a simulated fill field,
  labelled by the height-function method (heights are column sums of the
  fill level over 7 cells along the dominant normal axis, normal and
  curvature from their central differences); a sample is kept only when
  every one of its 3x3 columns starts in liquid and ends in gas.

This module only builds inputs; it contains none of the lattice method.
"""
from __future__ import annotations

import numpy as np

OFFS = np.array([(i % 3 - 1, (i // 3) % 3 - 1, i // 9 - 1) for i in range(27)], dtype=np.float64)


def _subpoints(ss):
    o = (np.arange(ss) + 0.5) / ss - 0.5
    g = np.stack(np.meshgrid(o, o, o, indexing="ij"), -1).reshape(-1, 3)
    return (OFFS[:, None, :] + g[None, :, :]).reshape(-1, 3)  # (27*ss^3, 3)


def _random_rotations(rng, m):
    q, r = np.linalg.qr(rng.standard_normal((m, 3, 3)))
    q = q * np.sign(np.diagonal(r, axis1=1, axis2=2))[:, None, :]
    det = np.linalg.det(q)
    q[det < 0, :, 0] *= -1
    return q


def _spheres(rng, m, P, ss):
    R = np.exp(rng.uniform(np.log(4.0), np.log(64.0), m))
    p0 = rng.uniform(-0.5, 0.5, (m, 3))
    d = rng.standard_normal((m, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    X = p0 - R[:, None] * d
    inside = ((P[None, :, :] - X[:, None, :]) ** 2).sum(-1) <= (R ** 2)[:, None]
    phi = inside.reshape(m, 27, ss ** 3).mean(-1)
    bubble = rng.random(m) < 0.5
    phi[bubble] = 1.0 - phi[bubble]
    out = -X / np.linalg.norm(X, axis=1, keepdims=True)   # from the centre towards the origin
    n = np.where(bubble[:, None], -out, out)
    kap = np.where(bubble, -1.0 / R, 1.0 / R)
    return phi, np.concatenate([n, kap[:, None]], axis=1)


def _sinusoids(rng, m, P, ss):
    lam = np.exp(rng.uniform(np.log(8.0), np.log(128.0), m))
    k = 2 * np.pi / lam
    rmin = np.exp(rng.uniform(np.log(4.0), np.log(64.0), m))
    A = np.minimum(1.0 / (rmin * k * k), 1.5 / k)           # slope at most 1.5
    psi = rng.uniform(0, 2 * np.pi, m)
    Q = _random_rotations(rng, m)                            # columns e1, e2, e3
    p0 = rng.uniform(-0.5, 0.5, (m, 3))
    s = np.einsum("mi,mi->m", p0, Q[:, :, 2]) - A * np.sin(k * np.einsum("mi,mi->m", p0, Q[:, :, 0]) + psi)
    u = np.einsum("pi,mi->mp", P, Q[:, :, 0])
    w = np.einsum("pi,mi->mp", P, Q[:, :, 2])
    liquid = w < A[:, None] * np.sin(k[:, None] * u + psi[:, None]) + s[:, None]
    phi = liquid.reshape(m, 27, ss ** 3).mean(-1)
    # nearest point of the curve w = h(u) to the origin (Newton on u + h h' = 0)
    uu = np.zeros(m)
    for _ in range(50):
        h = A * np.sin(k * uu + psi) + s
        h1 = A * k * np.cos(k * uu + psi)
        h2 = -A * k * k * np.sin(k * uu + psi)
        g = uu + h * h1
        gp = 1.0 + h1 * h1 + h * h2
        gp = np.where(np.abs(gp) < 1e-3, np.sign(gp) * 1e-3 + (gp == 0) * 1e-3, gp)
        uu = uu - np.clip(g / gp, -1.0, 1.0)
    h1 = A * k * np.cos(k * uu + psi)
    h2 = -A * k * k * np.sin(k * uu + psi)
    nrm = (-h1[:, None] * Q[:, :, 0] + Q[:, :, 2]) / np.sqrt(1 + h1 * h1)[:, None]
    kap = -h2 / (2.0 * (1 + h1 * h1) ** 1.5)                # mean curvature of a cylinder
    return phi, np.concatenate([nrm, kap[:, None]], axis=1)


def analytic_stencils(n: int, seed: int = 0, ss: int = 8, chunk: int = 256):
    """n stencils (fill levels, shape (n, 27)) and labels (n, 4)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    P = _subpoints(ss)
    xs, ys = [], []
    have = 0
    while have < n:
        m = min(chunk, 2 * (n - have) + 8)
        half = m // 2
        for fn, mm in ((_spheres, half), (_sinusoids, m - half)):
            phi, lab = fn(rng, mm, P, ss)
            ok = (phi[:, 13] > 0.0) & (phi[:, 13] < 1.0)
            xs.append(phi[ok])
            ys.append(lab[ok])
            have += int(ok.sum())
    X = np.concatenate(xs)[:n]
    Y = np.concatenate(ys)[:n]
    perm = rng.permutation(n)
    return X[perm], Y[perm]


def height_function_samples(types, fill, liquid=1, gas=0, interface=2, solid=3, max_samples=None,
                            seed: int = 0):
    """Height-function labelled stencils from a simulated field.

    types, fill: (nz, ny, nx) arrays of a lattice (x, y periodic; z walls).
    Returns (X (m, 27), Y (m, 4), cells (m,)) for the interface cells whose
    3x3 columns of 7 cells along the dominant normal axis all start in
    liquid (fill 1) and end in gas (fill 0)."""
    nz, ny, nx = types.shape
    phi = np.where(types == liquid, 1.0, np.where(types == interface, np.clip(fill, 0, 1), 0.0))
    solid_m = types == solid
    zz, yy, xx = np.nonzero(types == interface)
    keep = (zz >= 3) & (zz <= nz - 4)
    zz, yy, xx = zz[keep], yy[keep], xx[keep]

    def at(dz, dy, dx):
        return phi[zz + dz, (yy + dy) % ny, (xx + dx) % nx]

    def sol(dz, dy, dx):
        return solid_m[zz + dz, (yy + dy) % ny, (xx + dx) % nx]

    X = np.stack([at(int(o[2]), int(o[1]), int(o[0])) for o in OFFS], axis=1)
    anysolid = np.zeros(len(zz), bool)
    for o in OFFS:
        anysolid |= sol(int(o[2]), int(o[1]), int(o[0]))
    # dominant axis from the Parker-Youngs-free simple gradient of the stencil
    g = np.stack([(X[:, OFFS[:, d] == 1].sum(1) - X[:, OFFS[:, d] == -1].sum(1)) for d in range(3)], 1)
    axis = np.argmax(np.abs(g), axis=1)
    labels = np.full((len(zz), 4), np.nan)
    valid = ~anysolid
    for a in range(3):
        for sgn in (-1, 1):          # sgn = -1: liquid towards -axis (fill decreases along +axis)
            sel = valid & (axis == a) & (np.sign(g[np.arange(len(zz)), a]) == -sgn * 1) if False else None
            sel = valid & (axis == a) & (np.sign(g[:, a]) == (-1 if sgn == 1 else 1))
            if not sel.any():
                continue
            b_ax, c_ax = [d for d in range(3) if d != a]
            H = np.zeros((sel.sum(), 3, 3))
            good = np.ones(sel.sum(), bool)
            for ib, db in enumerate((-1, 0, 1)):
                for ic, dc in enumerate((-1, 0, 1)):
                    col = []
                    for t in range(-3, 4):
                        d = [0, 0, 0]
                        d[a] = sgn * t
                        d[b_ax] = db
                        d[c_ax] = dc
                        col.append(phi[(zz[sel] + d[2]), (yy[sel] + d[1]) % ny, (xx[sel] + d[0]) % nx])
                        good &= ~solid_m[(zz[sel] + d[2]), (yy[sel] + d[1]) % ny, (xx[sel] + d[0]) % nx]
                    col = np.stack(col, 1)   # from the liquid end to the gas end
                    good &= (col[:, 0] == 1.0) & (col[:, -1] == 0.0)
                    H[:, ib, ic] = col.sum(1) - 3.5
            hb = 0.5 * (H[:, 2, 1] - H[:, 0, 1])
            hc = 0.5 * (H[:, 1, 2] - H[:, 1, 0])
            hbb = H[:, 2, 1] - 2 * H[:, 1, 1] + H[:, 0, 1]
            hcc = H[:, 1, 2] - 2 * H[:, 1, 1] + H[:, 1, 0]
            hbc = 0.25 * (H[:, 2, 2] - H[:, 2, 0] - H[:, 0, 2] + H[:, 0, 0])
            q = 1 + hb * hb + hc * hc
            kap = -((1 + hc * hc) * hbb - 2 * hb * hc * hbc + (1 + hb * hb) * hcc) / (2 * q ** 1.5)
            n = np.zeros((sel.sum(), 3))
            n[:, a] = sgn
            n[:, b_ax] = -hb * sgn
            n[:, c_ax] = -hc * sgn
            n /= np.linalg.norm(n, axis=1, keepdims=True)
            lab = np.concatenate([n, kap[:, None]], 1)
            lab[~good] = np.nan
            labels[sel] = lab
    ok = np.all(np.isfinite(labels), axis=1)
    X, Y = X[ok], labels[ok]
    cells = (xx + nx * (yy + ny * zz))[ok]
    if max_samples is not None and len(X) > max_samples:
        idx = np.random.Generator(np.random.PCG64(seed)).choice(len(X), max_samples, replace=False)
        X, Y, cells = X[idx], Y[idx], cells[idx]
    return X, Y, cells
