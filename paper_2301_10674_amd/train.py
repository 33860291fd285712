"""Training data and driver of the learned interface estimator.

    python -m paper_2301_10674_amd.train [--analytic N] [--flume-steps S]
        [--every K] [--flume-samples M] [--epochs E] [--out weights.npy]

Data (90/10 split, seeded):

* analytic droplets, bubbles and sinusoidal sheets (``stencils.
  analytic_stencils``), generated in parallel chunks with per-chunk seeds;
* fill fields that the lattice itself produces on the flume, sampled every
  K steps and labelled by the height-function method (``stencils.
  height_function_samples``).

The network is trained on the GPU by the library's own kernels
(``fsl_estimator_train``) towards the corrections of the finite-difference
estimates (``fsl_fd_geometry``, see ``estimator``) and gated against the
finite-difference estimate on the held-out part: it is used only if it is
better in both RMS angle and RMS curvature error.
"""
from __future__ import annotations

import argparse
import json
import os
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

from . import estimator as E
from . import stencils as ST

LIQUID, INTERFACE, SOLID, GAS = 1, 2, 3, 0


def _analytic_chunk(args):
    n, seed, ss = args
    return ST.analytic_stencils(n, seed=seed, ss=ss)


def analytic_dataset(n, seed=0, ss=6, chunk=20000, workers=None):
    """n analytic stencils in chunks of `chunk`, chunk k drawn with seed
    (seed, k); the result does not depend on the number of workers."""
    jobs = [(min(chunk, n - a), int(np.random.SeedSequence([seed, k]).generate_state(1)[0]), ss)
            for k, a in enumerate(range(0, n, chunk))]
    workers = workers or min(16, os.cpu_count() or 1, len(jobs))
    if workers > 1:
        with ProcessPoolExecutor(workers) as ex:
            parts = list(ex.map(_analytic_chunk, jobs))
    else:
        parts = [_analytic_chunk(j) for j in jobs]
    return np.concatenate([p[0] for p in parts]), np.concatenate([p[1] for p in parts])


def analytic_dataset_gpu(fsl, n, seed=0, ss=16):
    """n analytic stencils with their fill levels supersampled on ss^3 points
    per cell on the GPU (fsl_estimator_stencils)."""
    return ST.analytic_stencils(n, seed=seed, ss=ss, fill=fsl.estimator_stencils)


def lattice_samples(lat, fsl):
    """Height-function labelled stencils of a lattice's current fill field."""
    f = lat.read_fields([fsl.FIELD_TYPE, fsl.FIELD_FILL])
    X, Y, cells = ST.height_function_samples(f[fsl.FIELD_TYPE], f[fsl.FIELD_FILL], liquid=LIQUID,
                                             gas=GAS, interface=INTERFACE, solid=SOLID)
    return X, Y, cells


def flume_dataset(lat, fsl, steps, every, max_samples, seed=0):
    """Step the lattice `steps` times, labelling its fill field every
    `every` steps; at most max_samples stencils, drawn without replacement."""
    xs, ys = [], []
    done = 0
    while done < steps:
        k = min(every, steps - done)
        lat.step(k)
        done += k
        X, Y, _ = lattice_samples(lat, fsl)
        xs.append(X)
        ys.append(Y)
    X, Y = np.concatenate(xs), np.concatenate(ys)
    if len(X) > max_samples:
        idx = np.random.Generator(np.random.PCG64(seed)).choice(len(X), max_samples, replace=False)
        X, Y = X[idx], Y[idx]
    return X, Y


def split(X, Y, val_frac=0.1, seed=0):
    perm = np.random.Generator(np.random.PCG64(seed)).permutation(len(X))
    nv = int(round(val_frac * len(X)))
    v, t = perm[:nv], perm[nv:]
    return X[t], Y[t], X[v], Y[v]


def evaluate(fsl, w, X, Y, fd=None):
    """(network errors, finite-difference errors) on (X, Y): RMS angle in
    degrees and RMS curvature error; the network corrects the finite-
    difference estimate of each stencil."""
    fd = np.asarray(fsl.fd_geometry(X), dtype=np.float64) if fd is None else fd
    net = E.compose(fsl.estimator_infer(w, X), fd)
    return E.errors(net, Y), E.errors(fd, Y)


def train(fsl, X, Y, Xv, Yv, epochs=20, batch=512, lr=2e-3, seed=0):
    """Train on (X, Y) towards the corrections of the finite-difference
    estimates (computed on the GPU), validate on (Xv, Yv)."""
    t0 = time.perf_counter()
    T = E.residual_targets(Y, fsl.fd_geometry(X))
    w, losses = fsl.estimator_train(X, T, E.init_weights(seed), epochs=epochs, batch=batch, lr=lr, seed=seed)
    secs = time.perf_counter() - t0
    net_err, fd_err = evaluate(fsl, w, Xv, Yv)
    return {"weights": w, "losses": [float(v) for v in losses], "train_seconds": secs,
            "train_samples": int(len(X)), "val_samples": int(len(Xv)),
            "net_err": net_err, "fd_err": fd_err, "gate": bool(E.gate(net_err, fd_err))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--analytic", type=int, default=500000)
    ap.add_argument("--flume-steps", type=int, default=2000)
    ap.add_argument("--every", type=int, default=100)
    ap.add_argument("--flume-samples", type=int, default=500000)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default="estimator_weights.npy")
    args = ap.parse_args()

    from . import fsl, inputs

    t0 = time.perf_counter()
    Xa, Ya = analytic_dataset(args.analytic, seed=args.seed)
    ta = time.perf_counter() - t0
    w = inputs.flume(seed=2)
    lat = fsl.lattice_from_workload(w, "fp32")
    t0 = time.perf_counter()
    Xf, Yf = flume_dataset(lat, fsl, args.flume_steps, args.every, args.flume_samples, seed=args.seed)
    tf = time.perf_counter() - t0
    lat.destroy()
    X, Y = np.concatenate([Xa, Xf]), np.concatenate([Ya, Yf])
    src = np.concatenate([np.zeros(len(Xa), bool), np.ones(len(Xf), bool)])
    Xt, Yt, Xv, Yv = split(X, Y, 0.1, seed=args.seed)
    _, st, _, sv = split(X, src, 0.1, seed=args.seed)   # the same permutation
    rep = train(fsl, Xt, Yt, Xv, Yv, epochs=args.epochs, seed=args.seed)
    # the two sources separately, on the held-out part
    rep["analytic_val"] = evaluate(fsl, rep["weights"], Xv[~sv], Yv[~sv])
    rep["flume_val"] = evaluate(fsl, rep["weights"], Xv[sv], Yv[sv])
    np.save(args.out, rep.pop("weights"))
    rep.update(analytic_samples=int(len(Xa)), flume_samples=int(len(Xf)), analytic_seconds=ta,
               flume_seconds=tf)
    print(json.dumps(rep))


if __name__ == "__main__":
    main()
