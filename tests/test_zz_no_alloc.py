"""The allocation-free gradient entry point (fsl_estimator_grad_device: every
array in device memory, the partial sums in the library's per-GPU scratch
array) against the allocating one (fsl_estimator_grad), through the C-ABI,
on two calls in a row, the second with fewer samples, so that a result
cannot lean on what the first call left in the scratch.

Both run the same kernels; only the grouping of the FP32 partial sums
differs (several sample groups per wavefront here, one there), so the
gradients agree to FP32 rounding of the summation order: 1e-5 relative
(norm) and the loss to 1e-5 relative.
"""
import numpy as np
import pytest

from paper_2301_10674_amd import estimator as E

pytestmark = pytest.mark.gpu


def F():
    from paper_2301_10674_amd import fsl
    return fsl


def batch(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.0, (n, 27)).astype(np.float32)
    y = (0.3 * rng.standard_normal((n, 4))).astype(np.float32)
    return x, y


def test_allocation_free_gradient_matches_the_allocating_one():
    import torch

    f = F()
    w = (E.init_weights(9) * 1.5).astype(np.float32)
    wt = torch.tensor(w, device="cuda")
    g = torch.empty(6212, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    for n, seed in ((9000, 1), (700, 2)):
        x, y = batch(n, seed)
        g_ref, loss_ref = f.estimator_grad(w, x, y)
        xt, yt = torch.tensor(x, device="cuda"), torch.tensor(y, device="cuda")
        g.fill_(float("nan"))
        loss.fill_(float("nan"))
        f.estimator_grad_device(wt, xt, yt, g, loss)
        torch.cuda.synchronize()
        gd, ld = g.cpu().numpy(), float(loss.cpu().numpy()[0])
        rel = np.linalg.norm(gd - g_ref) / np.linalg.norm(g_ref)
        print("n = %d: gradient relative difference %.2e, loss %.8g against %.8g" % (n, rel, ld, loss_ref))
        assert np.all(np.isfinite(gd)) and rel <= 1e-5
        assert abs(ld - loss_ref) <= 1e-5 * abs(loss_ref)


def test_allocation_free_gradient_rejects_bad_sizes():
    import torch

    f = F()
    t = torch.zeros(16, dtype=torch.float32, device="cuda")
    for n in (0, (1 << 24) + 1):
        with pytest.raises(f.FslError) as e:
            f.estimator_grad_device(t, t, t, t, t, n=n)
        assert "status 1" in str(e.value)
