"""Learned interface estimator: targets, composition and the gate.

The network, its loss, the training kernels and the inference inside the
lattice step live in the HIP library (``fsl_estimator_*``).  The network
reads the 3x3x3 fill stencil and predicts the correction to the finite-
difference estimate of the same stencil (Parker-Youngs normal n_fd and
Hessian curvature k_fd):

    n_raw = n_fd + y[0:3],  n = n_raw / |n_raw|,  kappa = k_fd + y[3] / 4,

so that planar interfaces, where finite differences are exact, stay exact,
and the curvature keeps the finite-difference response to the fill field.
This module prepares the training targets and initial weights, composes
predictions, and holds the validation gate:

* ``init_weights``: seeded Glorot-uniform weights, zero biases;
* ``residual_targets`` / ``compose``: labels -> network targets, network
  outputs -> (normal, curvature);
* ``errors``: RMS angle (degrees) and RMS curvature error of predictions;
* ``gate``: the network is used by a lattice only if it beats the finite-
  difference estimate on held-out data in both errors.
"""
from __future__ import annotations

import numpy as np

SHAPES = ((64, 27), (64,), (64, 64), (64,), (4, 64), (4,))


def init_weights(seed: int = 0) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for shp in SHAPES:
        if len(shp) == 2:
            lim = np.sqrt(6.0 / (shp[0] + shp[1]))
            parts.append(rng.uniform(-lim, lim, shp).ravel())
        else:
            parts.append(np.zeros(shp))
    return np.concatenate(parts).astype(np.float32)


def residual_targets(labels, fd):
    """Network targets: (n* - n_fd, kappa* - k_fd) for labels (n*, kappa*)
    and the finite-difference estimates fd, both (n, 4)."""
    labels = np.asarray(labels, dtype=np.float64)
    fd = np.asarray(fd, dtype=np.float64)
    return (labels - fd).astype(np.float32)


def compose(y, fd):
    """(normal, kappa) from raw network outputs y and the finite-difference
    estimates fd, both (n, 4)."""
    y = np.asarray(y, dtype=np.float64)
    fd = np.asarray(fd, dtype=np.float64)
    out = np.empty_like(y)
    n = fd[:, :3] + y[:, :3]
    out[:, :3] = n / np.maximum(np.linalg.norm(n, axis=1, keepdims=True), 1e-30)
    out[:, 3] = fd[:, 3] + 0.25 * y[:, 3]
    return out


def errors(pred, labels):
    """pred: (n, 4) = unnormalised normal + curvature; labels: (n, 4)."""
    n = pred[:, :3] / np.maximum(np.linalg.norm(pred[:, :3], axis=1, keepdims=True), 1e-30)
    cosang = np.clip((n * labels[:, :3]).sum(1), -1.0, 1.0)
    ang = np.degrees(np.arccos(cosang))
    return float(np.sqrt(np.mean(ang ** 2))), float(np.sqrt(np.mean((pred[:, 3] - labels[:, 3]) ** 2)))


def gate(net_err, fd_err):
    return net_err[0] < fd_err[0] and net_err[1] < fd_err[1]
