"""Training and test stencils for the learned interface estimator.

A sample is the 3x3x3 fill-level stencil around an interface cell (entry
k = a + 3b + 9c holds the cell at offset (a-1, b-1, c-1)) and a label: the
unit normal pointing from liquid to gas and the mean curvature kappa
(positive for convex liquid, so that 2 sigma kappa is the Laplace pressure
of Section 2.1).

* ``analytic_stencils``: seeded droplets / bubbles (radius log-uniform in
  [4, 64]) and sinusoidal sheets (minimum radius of curvature log-uniform in
  [4, 64], random orientation and phase); fill levels by supersampling each
  cell on an ss^3 grid (``fill_cpu``, or the library's
  ``fsl_estimator_stencils`` on the GPU for large sets at 16^3); labels
  exact at the surface point nearest to the centre of the stencil.
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


NPARAM = 16  # shape parameters per stencil, the layout of fsl_estimator_stencils


def _sphere_params(rng, m):
    """m droplets / bubbles: (params (m, 16), labels (m, 4))."""
    R = np.exp(rng.uniform(np.log(4.0), np.log(64.0), m))
    p0 = rng.uniform(-0.5, 0.5, (m, 3))
    d = rng.standard_normal((m, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    X = p0 - R[:, None] * d
    bubble = rng.random(m) < 0.5
    out = -X / np.linalg.norm(X, axis=1, keepdims=True)   # from the centre towards the origin
    n = np.where(bubble[:, None], -out, out)
    kap = np.where(bubble, -1.0 / R, 1.0 / R)
    prm = np.zeros((m, NPARAM))
    prm[:, 1] = bubble
    prm[:, 2:5] = X
    prm[:, 5] = R
    return prm, np.concatenate([n, kap[:, None]], axis=1)


def _sinusoid_params(rng, m):
    """m sinusoidal sheets: (params (m, 16), labels (m, 4))."""
    lam = np.exp(rng.uniform(np.log(8.0), np.log(128.0), m))
    k = 2 * np.pi / lam
    rmin = np.exp(rng.uniform(np.log(4.0), np.log(64.0), m))
    A = np.minimum(1.0 / (rmin * k * k), 1.5 / k)           # slope at most 1.5
    psi = rng.uniform(0, 2 * np.pi, m)
    Q = _random_rotations(rng, m)                            # columns e1, e2, e3
    p0 = rng.uniform(-0.5, 0.5, (m, 3))
    s = np.einsum("mi,mi->m", p0, Q[:, :, 2]) - A * np.sin(k * np.einsum("mi,mi->m", p0, Q[:, :, 0]) + psi)
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
    prm = np.zeros((m, NPARAM))
    prm[:, 0] = 1.0
    prm[:, 2:5] = Q[:, :, 0]
    prm[:, 5:8] = Q[:, :, 2]
    prm[:, 8], prm[:, 9], prm[:, 10], prm[:, 11] = A, k, psi, s
    return prm, np.concatenate([nrm, kap[:, None]], axis=1)


def fill_cpu(prm, ss):
    """Fill levels (m, 27) of shapes prm (m, 16) supersampled on ss^3 points
    per cell (the definition fsl_estimator_stencils evaluates on the GPU)."""
    P = _subpoints(ss)
    m = len(prm)
    out = np.empty((m, 27))
    sph = prm[:, 0] == 0.0
    if sph.any():
        q = prm[sph]
        d = P[None, :, :] - q[:, None, 2:5]
        r2 = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
        out[sph] = (r2 <= (q[:, 5] * q[:, 5])[:, None]).reshape(-1, 27, ss ** 3).mean(-1)
    if (~sph).any():
        q = prm[~sph]
        u = (P[None, :, 0] * q[:, None, 2] + P[None, :, 1] * q[:, None, 3]) + P[None, :, 2] * q[:, None, 4]
        w = (P[None, :, 0] * q[:, None, 5] + P[None, :, 1] * q[:, None, 6]) + P[None, :, 2] * q[:, None, 7]
        h = q[:, None, 8] * np.sin(q[:, None, 9] * u + q[:, None, 10]) + q[:, None, 11]
        out[~sph] = (w < h).reshape(-1, 27, ss ** 3).mean(-1)
    out = np.where(prm[:, 1:2] != 0.0, 1.0 - out, out)
    return out


def analytic_params(n, seed=0):
    """Shape parameters and labels of n candidate stencils, half droplets /
    bubbles and half sinusoidal sheets, in interleaved chunks."""
    rng = np.random.Generator(np.random.PCG64(seed))
    prms, labs = [], []
    have, chunk = 0, 4096
    while have < n:
        m = min(chunk, n - have + 1)
        half = m // 2
        for fn, mm in ((_sphere_params, half), (_sinusoid_params, m - half)):
            if mm:
                a, b = fn(rng, mm)
                prms.append(a)
                labs.append(b)
                have += mm
    return np.concatenate(prms)[:n], np.concatenate(labs)[:n]


def analytic_stencils(n: int, seed: int = 0, ss: int = 8, chunk: int = 256, fill=None):
    """n stencils (fill levels, shape (n, 27)) and labels (n, 4): shapes drawn
    until n of them have a partly filled centre cell.  fill(prm, ss) makes
    the fill levels (fill_cpu by default; the GPU's fsl_estimator_stencils
    gives the same values)."""
    fill = fill or fill_cpu
    rng = np.random.Generator(np.random.PCG64(seed))
    xs, ys = [], []
    have, rnd = 0, 0
    while have < n:
        want = int(1.3 * (n - have)) + 64
        prm, lab = analytic_params(want, seed=int(np.random.SeedSequence([seed, rnd]).generate_state(1)[0]))
        rnd += 1
        phi = np.asarray(fill(prm, ss), dtype=np.float64)
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
