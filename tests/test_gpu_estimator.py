"""GPU tests of the learned interface estimator (BF16 matrix-core kernels).

* gradient and inference agree with the FP64 oracle evaluated at the same
  BF16-rounded weights and inputs (the GPU also rounds activations to BF16,
  hence the 2e-2 relative tolerance);
* training lowers the loss;
* gain test: trained on seeded analytic stencils towards the corrections of
  the finite-difference estimate (Parker-Youngs normal, Hessian curvature;
  the oracle's), the corrected estimate beats the finite-difference one on
  held-out stencils in both RMS angle and RMS curvature error;
* a lattice with the estimator attached runs, uses the network and falls
  back where required, and still conserves mass.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2301_10674_amd import estimator as E
from paper_2301_10674_amd import inputs as I
from paper_2301_10674_amd import stencils as ST

pytestmark = pytest.mark.gpu


def F():
    from paper_2301_10674_amd import fsl
    return fsl


def bf16(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def net_input(x):
    return np.clip(x, 0.0, 1.0) - 0.5


@pytest.fixture(scope="module")
def data():
    X, Y = ST.analytic_stencils(40000, seed=11, ss=6)
    Xh, Yh = ST.analytic_stencils(4000, seed=12, ss=6)
    return X, Y, Xh, Yh


def test_gradient_matches_oracle(data):
    X, Y = data[0][:512], data[1][:512]
    w = bf16(E.init_weights(3) * 1.5)
    xr = bf16(net_input(X)) + 0.5          # GPU input after its own rounding
    g_gpu, loss_gpu = F().estimator_grad(w, xr, Y)
    loss_cpu, g_cpu = O.mlp_loss_grad(w.astype(np.float64), bf16(net_input(X)).astype(np.float64), Y)
    assert abs(loss_gpu - loss_cpu) <= 1e-2 * loss_cpu
    rel = np.linalg.norm(g_gpu - g_cpu) / np.linalg.norm(g_cpu)
    assert rel <= 2e-2, rel
    # every parameter block carries gradient
    offs = [0, 1728, 1792, 5888, 5952, 6208, 6212]
    for a, b in zip(offs[:-1], offs[1:]):
        blk = np.linalg.norm(g_gpu[a:b] - g_cpu[a:b]) / max(np.linalg.norm(g_cpu[a:b]), 1e-12)
        assert blk <= 5e-2, (a, b, blk)


def test_inference_matches_oracle(data):
    X = data[0][:1000]
    w = bf16(E.init_weights(4) * 1.5)
    y_gpu = F().estimator_infer(w, bf16(net_input(X)) + 0.5)
    y_cpu = O.mlp_forward(w.astype(np.float64), bf16(net_input(X)).astype(np.float64))
    rel = np.linalg.norm(y_gpu - y_cpu) / np.linalg.norm(y_cpu)
    assert rel <= 2e-2, rel


def test_training_lowers_loss(data):
    X, Y = data[0][:8192], data[1][:8192]
    w0 = E.init_weights(5)
    w, losses = F().estimator_train(X, Y, w0, epochs=6, batch=256, lr=2e-3, seed=1)
    assert np.all(np.isfinite(losses)) and np.all(np.isfinite(w))
    assert losses[-1] < 0.5 * losses[0], losses
    _, l0 = F().estimator_grad(w0, X, Y)
    _, l1 = F().estimator_grad(w, X, Y)
    assert l1 < 0.5 * l0


def fd_predictions(X):
    out = np.zeros((len(X), 4))
    for i, s in enumerate(X):
        n, k = O.normal_curvature(np.clip(s, 0, 1))
        out[i, :3] = n
        out[i, 3] = k
    return out


def test_network_beats_finite_differences(data):
    X, Y, Xh, Yh = data
    T = E.residual_targets(Y, fd_predictions(X))
    w, losses = F().estimator_train(X, T, E.init_weights(6), epochs=25, batch=512, lr=2e-3, seed=2)
    fd = fd_predictions(Xh)
    net = E.compose(F().estimator_infer(w, Xh), fd)
    e_net, e_fd = E.errors(net, Yh), E.errors(fd, Yh)
    print("held-out RMS angle / kappa error: network %.2f deg / %.4f, finite differences %.2f deg / %.4f"
          % (e_net[0], e_net[1], e_fd[0], e_fd[1]))
    assert E.gate(e_net, e_fd)


def test_lattice_with_estimator_conserves_mass(data):
    X, Y = data[0][:20000], data[1][:20000]
    T = E.residual_targets(Y, fd_predictions(X))
    w, _ = F().estimator_train(X, T, E.init_weights(7), epochs=10, batch=512, lr=2e-3, seed=3)
    f = F()
    wl = I.channel_film()
    g = f.lattice_from_workload(wl, "fp32", normals=1)
    g.set_estimator(w)
    M0 = g.total_mass()
    g.step(100)
    used, fell = g.estimator_stats()
    assert used > 0
    assert abs(g.total_mass() - M0) <= 1e-12 * M0
    n = g.read(f.FIELD_NORMAL)
    t = g.read(f.FIELD_TYPE)
    itf = t == f.INTERFACE
    nn = np.linalg.norm(n[:, itf], axis=0)
    assert np.all((np.abs(nn - 1.0) < 1e-5) | (nn == 0.0))


def test_gpu_finite_differences_match_oracle(data):
    X = data[2][:2000]
    g = F().fd_geometry(X)
    o = fd_predictions(X)
    assert np.abs(g - o).max() < 1e-6
