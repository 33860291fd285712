"""Training driver of the learned interface estimator.

The network, its loss, the training kernels and the inference inside the
lattice step live in the HIP library (``fsl_estimator_*``); this module only
prepares data, initial weights and the validation gate:

* ``init_weights``: seeded Glorot-uniform weights, zero biases, except that
  the output bias starts the normal at +z (so |n_raw| > 0 from the start);
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
    w = np.concatenate(parts).astype(np.float32)
    w[-2] = 1.0   # b3[2]: start the normal at +z
    return w


def errors(pred, labels):
    """pred: (n, 4) = unnormalised normal + curvature; labels: (n, 4)."""
    n = pred[:, :3] / np.maximum(np.linalg.norm(pred[:, :3], axis=1, keepdims=True), 1e-30)
    cosang = np.clip((n * labels[:, :3]).sum(1), -1.0, 1.0)
    ang = np.degrees(np.arccos(cosang))
    return float(np.sqrt(np.mean(ang ** 2))), float(np.sqrt(np.mean((pred[:, 3] - labels[:, 3]) ** 2)))


def network_outputs(y):
    """Raw network outputs -> (normal, kappa) columns (output 3 is 4 kappa)."""
    out = np.array(y, dtype=np.float64)
    out[:, 3] *= 0.25
    return out


def gate(net_err, fd_err):
    return net_err[0] < fd_err[0] and net_err[1] < fd_err[1]
